/*
 * rfi.h -- C ABI of librfi, an MI355X (gfx950) implementation of the online,
 * post-correlation RFI screen of Yatawatta, Boonstra & Broekema, "Energy and
 * polarization based online interference mitigation in radio interferometry"
 * (arXiv 2412.14775).
 *
 * Problem statement (Section 2): N dual-polarised receivers give N(N+1)/2
 * baseline streams (autocorrelations included).  Each stream carries, per
 * channel and time sample i, the 2x2 correlation matrix
 *     V_i = [[xx_i, xy_i], [yx_i, yy_i]]                       (Section 2, eq. V)
 * and every stream is screened separately.  For each window of W samples the
 * screen forms complex Stokes I = xx+yy, Q = xx-yy, U = xy+yx, V = j(xy-yx)
 * (eq. IQUV), the spectral-kurtosis statistic of |I| (Section 2.1, Table 1)
 * and the directional statistic of the real and the imaginary parts of
 * (Q, U, V) (Section 2.2, Table 2), flags the window when a statistic leaves
 * its range (the tests are ORed), and leaves flagged windows out of the time
 * average, whose weight is updated (Section 2.1).
 *
 * Conventions for every entry point
 *  - Pointers named as device pointers must be device memory on the plan's
 *    device (HIP/PyTorch allocations); the caller owns every I/O buffer.
 *  - Functions return RFI_OK (0) or a negative rfi_status.  On error a message
 *    is available from rfi_last_error() (thread-local) and no output is
 *    written.  Invalid arguments are rejected before any device call.
 *  - No C++ exception crosses this boundary.
 *  - rfi_screen is asynchronous: it enqueues kernels on the caller's HIP
 *    stream and returns; the caller synchronises before reading outputs.
 */
#ifndef RFI_H
#define RFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RFI_ABI_VERSION 1

typedef enum rfi_status {
  RFI_OK = 0,
  RFI_ERR_INVALID_ARGUMENT = -1, /* bad shape, threshold, pointer or alignment          */
  RFI_ERR_OUT_OF_MEMORY = -2,    /* device allocation failed                             */
  RFI_ERR_DEVICE = -3,           /* a HIP call failed; the message holds HIP's error     */
  RFI_ERR_UNSUPPORTED = -4       /* valid request the library does not implement         */
} rfi_status;

/* Storage format of the visibilities.  Arithmetic is FP32 for both. */
typedef enum rfi_vis_format {
  RFI_VIS_CF32 = 0, /* complex64: per sample 4 x (re, im) float32, 32 bytes        */
  RFI_VIS_CF16 = 1  /* complex half: per sample 4 x (re, im) float16, 16 bytes     */
} rfi_vis_format;

/* Option bits of rfi_params.options. */
enum {
  RFI_OPT_NO_SK = 1u,   /* do not apply the spectral-kurtosis test (bits 0-1 cleared)  */
  RFI_OPT_NO_DS = 2u,   /* do not apply the directional test (bits 2-3 cleared)        */
  RFI_OPT_ADAPTIVE = 4u, /* per-stream thresholds from running null statistics, below   */
  RFI_OPT_PAPER_MIXED = 8u /* the paper's trained mixed precision (Tables 3-4): unit-vector  */
                           /* sums, their squares, r and the SK ratio in FP16 (binary16     */
                           /* rounding per operation), the rest FP32; complex64 storage and */
                           /* M = K S with K <= 8, S a power of two, F S <= 64 only         */
};

/* Flag bits written per window.  A window is flagged when any bit is set. */
enum {
  RFI_FLAG_SK_LOW = 1u,  /* not (tau >= s_low)      Section 2.1                  */
  RFI_FLAG_SK_HIGH = 2u, /* tau > s_high            Section 2.1                  */
  RFI_FLAG_DS_RE = 4u,   /* not (r_re <= gamma)     Section 2.2, real parts      */
  RFI_FLAG_DS_IM = 8u    /* not (r_im <= gamma)     Section 2.2, imaginary parts */
};

/*
 * Screen parameters: the problem statement of Section 2 and the
 * hyperparameters of Section 2.3 (d, s_low, s_high, gamma, W), fixed a priori.
 */
typedef struct rfi_params {
  int32_t n_stations;  /* N >= 1                                                          */
  int32_t n_baselines; /* must equal N(N+1)/2: pairs (p,q), p <= q, row-major upper triangle */
  int32_t n_channels;  /* C >= 1                                                          */
  int32_t n_samples;   /* T, time samples per integration; T % block_m == 0               */
  int32_t block_m;     /* M, window length in time samples (the paper's W when F = 1), >= 2 */
  int32_t vis_format;  /* rfi_vis_format                                                  */
  float sk_d;          /* d > 0 (Section 2.1)                                              */
  float sk_low;        /* s_low < s_high (Section 2.1)                                     */
  float sk_high;
  float ds_gamma;      /* gamma in [0, 1] (Section 2.2)                                    */
  float eps;           /* epsilon of Tables 1-2 (S1^2 + eps, sqrt(.) + eps); >= 0, finite  */
  uint32_t options;    /* RFI_OPT_* bits                                                   */
  float kappa_sk;      /* ADAPTIVE: s_low/high = mean_tau -/+ kappa_sk * sd_tau, kappa >= 0 */
  float kappa_ds;      /* ADAPTIVE: gamma_re/im = mean_r + kappa_ds * sd_r                  */
  int32_t n_warm;      /* ADAPTIVE: windows a stream must have seen before its own thresholds */
  int32_t block_f;     /* F, adjacent channels per window: 1 (time only), 2 or 4 (time x  */
                       /* frequency window of M x F samples, Sections 3.2 and 4.1)          */
} rfi_params;

typedef struct rfi_plan rfi_plan; /* opaque */

/* Fill *p with defaults: eps = 2^-23, d = 1, s_low = 0.5, s_high = 2, gamma = 0.4, M = 64,
 * block_f = 1, kappa_sk = kappa_ds = 3, n_warm = 0, CF32, options 0; sizes zero. */
void rfi_params_default(rfi_params *p);

/*
 * Validate *params, choose the kernel for (vis_format, block_m, block_f), and allocate
 * the plan's device state on `device` (the ADAPTIVE state, zeroed; nothing
 * otherwise).  On success *out receives the plan; on error *out is NULL.
 * Every M >= 2 and F in {1, 2, 4} is screened; the kernel depends on the shape: M a
 * power of two <= 4096 (F = 1); windows cut into F ceil(M / C) <= 64 runs of C <= 8
 * samples, one per lane; M of more than 128 (complex64) / 256 (complex half) samples
 * (F = 1); wider time x frequency windows (F > 1) over several steps of one channel's
 * chunk each.
 * Errors: INVALID_ARGUMENT (shape or threshold rules above), UNSUPPORTED (block_f not
 * 1, 2 or 4; RFI_OPT_PAPER_MIXED outside its shapes), DEVICE, OUT_OF_MEMORY.
 */
int rfi_plan_create(const rfi_params *params, int device, rfi_plan **out);

/*
 * Screen one integration (Sections 2.1-2.2).  All pointers are device pointers.
 *   vis    [B][C][T][4] samples in the plan's format, pol order (xx, xy, yx, yy),
 *          (re, im) interleaved; 16-byte aligned.                       (read)
 *   avg    [B][C][4][2] float32: flag-masked time average of each correlation
 *          over unflagged samples; 0 when every window is flagged.       (write)
 *   weight [B][C] float32: unflagged fraction of the T samples.           (write)
 *   flags  [B][C/F][T/M] uint8 RFI_FLAG_* bits per window, or NULL.       (write)
 *   stats  [B][C/F][T/M][3] float32 (tau, r_re, r_im) per window, or NULL.(write)
 * A window is M time samples of F adjacent channels (channels f*F .. f*F+F-1 of
 * one baseline); W = M F enters tau and r, and a flag removes the window's
 * samples of all F channels from their averages.
 *   hip_stream: a hipStream_t (NULL = default stream).
 * With RFI_OPT_ADAPTIVE the thresholds of each stream come from the plan's
 * state, which this call then updates from the unflagged windows; calls on one
 * plan must therefore be ordered (one stream at a time).  Buffers must not alias.
 * Asynchronous; errors: INVALID_ARGUMENT (NULL or misaligned pointer), DEVICE.
 */
int rfi_screen(rfi_plan *plan, const void *vis, float *avg, float *weight, uint8_t *flags,
               float *stats, void *hip_stream);

/* Free the plan and its device state.  NULL-safe.  Waits for nothing: the caller
 * must not destroy a plan with work in flight. */
int rfi_destroy(rfi_plan *plan);

/* Message of the last failed call on this thread ("" if none).  Valid until the
 * next call on this thread. */
const char *rfi_last_error(void);

/*
 * Device bytes one rfi_screen call of this plan touches or owns: the plan's
 * own state plus vis, avg, weight and flags (stats excluded).  Used for
 * admission control by memory footprint.
 */
int rfi_plan_footprint(const rfi_plan *plan, size_t *bytes);

/*
 * ADAPTIVE state, per channel group b*(C/F) + c/F (per stream when F = 1), 64 bytes:
 *   uint64 n; double mean[3]; double m2[3]; uint64 reserved
 * (statistics in the order tau, r_re, r_im; n = clean windows so far, exact; m2 = sum of
 * squared deviations).  Each call merges its integration's moments into it in float64
 * (Chan, Golub & LeVeque 1979): a float32 state would drift from the exact running values
 * by more than 1e-5 relative within 1e4-1e5 integrations.
 * rfi_state_get / rfi_state_set copy the whole state to / from host memory
 * synchronously (checkpoint / resume); bytes must equal rfi_state_bytes().
 * rfi_state_reset zeroes it on the given stream (one kernel, no memset node, so the
 * reset may be captured into a graph).
 */
size_t rfi_state_bytes(const rfi_plan *plan);
int rfi_state_get(rfi_plan *plan, void *host_dst, size_t bytes);
int rfi_state_set(rfi_plan *plan, const void *host_src, size_t bytes);
int rfi_state_reset(rfi_plan *plan, void *hip_stream);

/*
 * Read-only streaming probe: reads `bytes` (multiple of 16) from device buffer
 * `src` once and writes one float per workgroup into `sink` (device, at least
 * rfi_probe_sink_floats(bytes) floats) so the reads cannot be elided.
 * Gives the achievable HBM read bandwidth that bounds rfi_screen.
 */
size_t rfi_probe_sink_floats(size_t bytes);
int rfi_probe_read(const void *src, size_t bytes, float *sink, void *hip_stream);

/* Plain device copy of `bytes` (multiple of 16): a kernel of known traffic used to
 * calibrate hardware byte counters. */
int rfi_probe_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Device check of the complex-half sample sums: the windowed and long-window kernels form
 * the sums and differences of binary16 parts in one v_fma_mix_f32 each, which must equal
 * conversion to float32 followed by a float32 add, bit for bit.  Every binary16 value a is
 * taken against 1024 values b (signed zeros, subnormals, the largest finite values,
 * infinities, a NaN, pseudo-random patterns) in each form the kernels use; mismatches[a]
 * (device, 65536 uint32, written by the call) counts the differences, NaN results comparing
 * equal.  All zero means the kernels' complex-half sums are those of the plain definition.
 * Asynchronous on hip_stream.  Errors: RFI_ERR_INVALID_ARGUMENT for NULL. */
int rfi_probe_half_sums(uint32_t *mismatches, void *hip_stream);

/* ------------------------------------------------------------------------------------------
 * Hyperparameters (Section 2.3): the thresholds follow from a desired false-alarm
 * probability, and small windows need fine-tuning on RFI-free data.  Host functions, no
 * device access.
 * ------------------------------------------------------------------------------------------ */

/* Exact mean, variance and skewness of tau for i.i.d. Gamma(d)-distributed |I| in a window
 * of W samples (the null model of the SK estimator; mean 1, variance
 * 2d(d+1)W^2 Gamma(Wd+2) / ((W-1) Gamma(Wd+4))), from moments of the Dirichlet distribution
 * of |I_i| / S1.  Errors: INVALID_ARGUMENT (W < 2, d <= 0, NULL output). */
int rfi_sk_null_moments(int32_t W, float d, double *mean, double *var, double *skew);

/* Thresholds for false-alarm probabilities pfa_sk (two-sided, pfa/2 per side) and pfa_ds:
 * sk_low / sk_high = Cornish-Fisher quantiles of tau from its exact null moments; ds_gamma =
 * sqrt(chi2_3^-1(1 - pfa_ds) / (3W)) (3 W r^2 tends to chi-square with 3 degrees of freedom
 * for isotropic directions).  Approximate for small W (tau's lower tail especially); refine
 * with rfi_calibrate_from_stats.  W is the window size M F. */
int rfi_thresholds_from_pfa(int32_t W, float d, double pfa_sk, double pfa_ds, float *sk_low, float *sk_high,
                            float *ds_gamma);

/* Calibrate on the statistics of RFI-free data: `stats` is host memory [n_windows][3]
 * (tau, r_re, r_im) as rfi_screen writes them with sk_d = d_used.  d_cal makes the mean of tau
 * 1; sk_low / sk_high are the pfa_sk/2 and 1 - pfa_sk/2 quantiles of tau recomputed with
 * d_cal; ds_gamma is the 1 - pfa_ds quantile of the pooled r_re and nonzero r_im.  Non-finite
 * statistics are ignored.  Errors: INVALID_ARGUMENT (NULL, bad probabilities, degenerate data). */
int rfi_calibrate_from_stats(const float *stats, size_t n_windows, int32_t W, float d_used, double pfa_sk,
                             double pfa_ds, float *d_cal, float *sk_low, float *sk_high, float *ds_gamma);

/* ------------------------------------------------------------------------------------------
 * Serving: a persistent request loop that screens integrations of many arrays as they
 * arrive (continuous batching).  Not a paper passage: it serves the online use the paper
 * targets (Section 1: real time, before averaging, in the correlator).
 *
 * A request names a plan (one per array stream; its adaptive state lives on the device)
 * and that integration's device buffers, plus an arrival time on the server clock.  A
 * scheduler thread releases requests at their arrival time into a FIFO queue and admits
 * a request when (a) a slot (one HIP stream each) is free, (b) the footprint of all
 * admitted requests plus this one's (rfi_plan_footprint, plus the statistics output
 * [B][C/F][T/M][3] float32 when the request writes it) stays within the HBM budget, and
 * (c) no earlier request of the same plan is still queued or running (per-plan order keeps
 * the adaptive state update sequence of that array).  A request that cannot be admitted
 * does not block later requests of other plans.  Each admitted request replays a hipGraph
 * of its screen step (captured on first use for that plan and buffer set) on its slot's
 * stream; a host callback timestamps completion.  Requests of different arrays therefore
 * overlap on the device, and each result is bitwise the same as when run alone.  Graphs
 * are cached per plan identity, not per plan address: a plan created after another was
 * destroyed never replays the old plan's graph, even at the same address.  The cache holds
 * at most max_graphs graphs; when it is full the least recently used graph that no request
 * on the device replays is freed (graphs of destroyed plans and of buffer sets no longer
 * used age out this way), so a long run with fresh buffers stays bounded.  A failed
 * request completes with its status in rfi_completion.status; its message is recorded on
 * the scheduler thread, so rfi_last_error on the caller's thread does not show it.
 * ------------------------------------------------------------------------------------------ */
typedef struct rfi_server rfi_server; /* opaque */

typedef struct rfi_server_config {
  int32_t device;          /* HIP device                                                      */
  int32_t n_slots;         /* requests on the device at once (HIP streams), 1..64               */
  uint64_t hbm_budget;     /* bytes: cap on the summed footprint of admitted requests, > 0      */
  int32_t use_graphs;      /* 1: replay captured hipGraphs; 0: launch rfi_screen directly       */
  int32_t max_graphs;      /* graphs kept cached at most (0: 256); the least recently used one
                              that no request on the device replays is freed first               */
} rfi_server_config;

typedef struct rfi_request {
  rfi_plan *plan;          /* not owned; must outlive the request                               */
  const void *vis;         /* device buffers as for rfi_screen (flags / stats may be NULL)      */
  float *avg;
  float *weight;
  uint8_t *flags;
  float *stats;
  double arrival;          /* server clock, seconds (rfi_server_now); past values = now         */
  uint64_t tag;            /* caller's identifier, returned in the completion                   */
} rfi_request;

typedef struct rfi_completion {
  uint64_t tag;
  int32_t status;          /* RFI_OK or the error of the launch                                 */
  int32_t slot;            /* slot (stream) the request ran on                                  */
  double arrival;          /* server clock, seconds                                             */
  double admitted;         /* when the scheduler launched it                                    */
  double done;             /* when the device finished it (host callback)                       */
} rfi_completion;

typedef struct rfi_server_stats {
  uint64_t submitted, completed, failed;
  uint64_t peak_inflight_bytes;  /* largest summed footprint of admitted requests                */
  int32_t peak_inflight;         /* largest number of requests on the device at once            */
  int32_t graphs;                /* graphs captured so far                                      */
  int32_t graphs_cached;         /* graphs held in the cache now (<= max_graphs unless every
                                    cached graph was on the device when a new one was needed) */
} rfi_server_stats;

/* Create the server and start its scheduler thread.  Errors: INVALID_ARGUMENT, DEVICE. */
int rfi_server_create(const rfi_server_config *cfg, rfi_server **out);
/* Seconds since the server was created (monotonic clock). */
double rfi_server_now(const rfi_server *srv);
/* Queue a request (thread-safe; returns at once).  INVALID_ARGUMENT if a pointer is NULL or
 * the request's footprint alone exceeds the budget (the request could never be admitted).
 * The plan must stay alive (not rfi_destroy'ed) until the request's completion is polled.
 * The server's streams wait on no other stream: the input must be complete in device memory
 * when the request is submitted (synchronize the stream that produced it first), and the
 * buffers must stay untouched until the request's completion has been polled. */
int rfi_server_submit(rfi_server *srv, const rfi_request *req);
/* Move up to `max` completions into `out` (*n_out of them), waiting up to timeout_s seconds
 * for at least one.  Completions are returned in the order the device finished them. */
int rfi_server_poll(rfi_server *srv, rfi_completion *out, int32_t max, int32_t *n_out, double timeout_s);
/* Block until every submitted request has completed (or timeout_s passes: then DEVICE). */
int rfi_server_drain(rfi_server *srv, double timeout_s);
int rfi_server_get_stats(const rfi_server *srv, rfi_server_stats *out);
/* Stop the scheduler after draining, free streams and graphs.  NULL-safe. */
int rfi_server_destroy(rfi_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* RFI_H */
