/*
 * ksum -- sliced fast kernel summation on AMD MI355X (gfx950).
 *
 * Computes s_m = sum_{n=1}^{N} w_n K(x_n, y_m), m = 1..M, for radial kernels
 * K(x, y) = F(||x - y||) on R^d, by the slicing method of Hertrich, "Fast Kernel
 * Summation in High Dimensions via Slicing and Fourier Transforms":
 *
 *   s_m ~= (1/P) sum_p t_{m,p},  t_{m,p} = sum_n w_n k(<xi_p, x_n>, <xi_p, y_m>)
 *
 * (Algorithm "Sliced Fast Fourier Summation", Sec. 3), where k(s,t) = f(|s-t|)
 * is the one-dimensional counterpart of K (Table "tab:kernels") and xi_p are
 * random directions on the sphere.  The 1-D sums use
 *   - fast Fourier summation (Sec. 3.1) with direct transforms (NDFT) or the
 *     non-equispaced FFT (NFFT) for the Gaussian,
 *   - sorting + prefix sums (Sec. 3.2, Algorithm "fastsum_energy") for the
 *     negative distance kernel,
 *   - both, after splitting K = K1 + K2 (Sec. 3.3), for the Laplacian.
 *
 * Conventions shared by every entry point
 *   - Array arguments named x, y, w, s, grad_* and ws are HIP *device* pointers
 *     owned by the caller; a plan owns its own device tables.  Host pointers are
 *     named host_* or are documented as host memory.
 *   - Points are row-major and contiguous: x is N x d, y is M x d.
 *   - Calls that take a stream are asynchronous on that stream (a hipStream_t
 *     passed as void*, NULL = the null stream); argument errors are reported
 *     synchronously by the return value, device faults surface as KSUM_EDEVICE
 *     at a later call that synchronises.
 *   - No entry point aborts or throws; no entry point that takes a workspace
 *     allocates device memory.  ksum_last_error() describes the last failure of
 *     the calling thread.
 *   - A plan is immutable after creation; concurrent ksum_execute calls on one
 *     plan need distinct workspaces.
 */
#ifndef KSUM_H
#define KSUM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ksum_plan ksum_plan;

/* Kernels (Table "tab:kernels").  sigma is the Gaussian bandwidth,
 * K = exp(-||x-y||^2 / (2 sigma^2)); the Laplacian is K = exp(-alpha ||x-y||)
 * with alpha = 1/sigma; the negative distance kernel is K = -||x-y||; the Matern
 * kernel with nu = 3/2 is K = (1 + sqrt(3) r/beta) exp(-sqrt(3) r/beta), r = ||x-y||,
 * beta = sigma (1-D counterpart: the 1F2 form of the appendix on the Matern and
 * Laplacian kernels; Fourier summation by NFFT as in the paper's experiments). */
typedef enum {
  KSUM_GAUSSIAN = 1,
  KSUM_LAPLACIAN = 2,
  KSUM_NEGDIST = 3,
  KSUM_MATERN = 4
} ksum_kernel;

/* One-dimensional summation method.  AUTO picks NDFT for the Gaussian with at
 * most 64 coefficients and NFFT above, NFFT (smooth part) + SORT for the
 * Laplacian and SORT for the negative distance. */
typedef enum {
  KSUM_1D_AUTO = 0,
  KSUM_1D_NDFT = 1,
  KSUM_1D_NFFT = 2,
  KSUM_1D_SORT = 3
} ksum_method;

/* Arithmetic of the projection GEMM (the first step of Algorithm "Sliced Fast
 * Fourier Summation").  FP32 uses the FP32 matrix cores.  SPLIT_BF16 splits every
 * FP32 operand a into a_hi = bf16(a) and a_lo = bf16(a - a_hi) (round to nearest
 * even) and takes a product as a_hi b_hi + a_hi b_lo + a_lo b_hi on the BF16 matrix
 * cores with FP32 accumulation: each product is within about 2^-16 of the FP32
 * product.  Everything after the projection is the same FP32 / FP64 arithmetic in
 * both modes. */
typedef enum {
  KSUM_FP32 = 0,
  KSUM_SPLIT_BF16 = 1
} ksum_precision;

typedef enum {
  KSUM_OK = 0,
  KSUM_EINVAL = 1,        /* invalid argument (null pointer, size <= 0, bad parameter) */
  KSUM_EUNSUPPORTED = 2,  /* valid but not supported (e.g. a method the kernel cannot use) */
  KSUM_ENOMEM = 3,        /* device or host allocation failed at plan time */
  KSUM_EWORKSPACE = 4,    /* workspace smaller than ksum_workspace_size() */
  KSUM_ENONFINITE = 5,    /* an input holds a NaN or an infinity (only with params.check_finite) */
  KSUM_EDEVICE = 6        /* HIP runtime error, or no usable device */
} ksum_status;

/* Plan parameters.  Fill with ksum_params_default(), then override fields.
 *   sigma       kernel scale (> 0; Gaussian bandwidth, Laplacian 1/alpha; unused for NEGDIST)
 *   seed        seed of the direction generator (see ksum_generate_directions)
 *   directions  optional host array P*d (FP64, row p = xi_p, unit norm) used instead
 *               of the generator; copied at plan creation; may be NULL
 *   n_coeff     Fourier coefficients (defaults: Gaussian 64, Laplacian 256, Matern 1024):
 *               NDFT uses k = -n_coeff/2..n_coeff/2, NFFT the
 *               index set -n_coeff/2..n_coeff/2-1 with the coefficient at -n_coeff/2
 *               set to 0 (so the sum stays real); even, 2..4096
 *   coeff_eps   cutoff of eq. "Fourier_cutoff": coefficients with |c_k| <= eps are dropped
 *   T           rescaling threshold of Sec. 3.1, 0 < T < 0.25 (0 = method default:
 *               Gaussian NDFT 0.045, Gaussian NFFT 0.02, Laplacian and Matern 0.125)
 *   oversample  NFFT grid oversampling (2 or 4); grid size n = oversample * n_coeff
 *   window_m    NFFT Kaiser-Bessel window half-width in grid cells (2..8)
 *   method      ksum_method
 *   precision   ksum_precision
 *   slice_batch slices per batch B (0 = all P); bounds the workspace (Remark on
 *               memory requirements and batching, Sec. 4.4)
 *   device      HIP device ordinal the plan is created on
 *   check_finite 1: ksum_execute*, ksum_execute_noalloc and ksum_backward first pass once
 *               over their inputs (x, y, w and grad_s) and wait for the result; a NaN or
 *               an infinity makes the call return KSUM_ENONFINITE before any other work,
 *               with no output written.  The wait makes such calls synchronous with
 *               their stream.  0 (default): no check; a non-finite input gives
 *               unspecified results (the sort places a NaN projection last). */
typedef struct {
  double sigma;
  uint64_t seed;
  const double *directions;
  int32_t n_coeff;
  double coeff_eps;
  double T;
  int32_t oversample;
  int32_t window_m;
  int32_t method;
  int32_t precision;
  int32_t slice_batch;
  int32_t device;
  int32_t check_finite;
} ksum_params;

/* Optional intermediate outputs of ksum_execute_probe (each pointer may be NULL).
 *   z      device float[P][M+N]: projections <xi_p, .>, targets first, then sources
 *   bounds device double[P][2]: c_min, c_max of each slice (the FP32 values used)
 *   t      device float[P][M]: the per-slice 1-D sums t_{m,p}
 *   perm   device int32[P][M+N]: the stable ascending order of each slice's
 *          projections (union index: 0..M-1 targets, M..M+N-1 sources); only
 *          produced by methods that sort (NEGDIST, LAPLACIAN) */
typedef struct {
  float *z;
  double *bounds;
  float *t;
  int32_t *perm;
} ksum_probe;

/* Library version string. */
const char *ksum_version(void);

/* Human-readable name of a status code (static storage). */
const char *ksum_status_string(ksum_status status);

/* Message describing the last failed call on the calling thread ("" if none). */
const char *ksum_last_error(void);

/* Default parameters for a kernel (host only, no device access).
 * EINVAL if out is NULL or kernel is unknown. */
ksum_status ksum_params_default(ksum_kernel kernel, ksum_params *out);

/* Validate (d, P, kernel, params) exactly as ksum_plan_create does, without
 * touching a device.  Returns KSUM_OK or the status plan creation would return. */
ksum_status ksum_check_params(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params);

/* Draw P directions uniform on S^{d-1} into host_out (host, FP64, P*d, row-major).
 * The first step of Algorithm "Sliced Fast Fourier Summation" leaves the
 * generator open; this one is: SplitMix64 (Steele, Lea, Flood 2014) output number
 * c of seed s is mix(s + (c+1)*0x9E3779B97F4A7C15); coordinate i of direction p
 * takes outputs c = 2(p*d+i) and c+1, u1 = ((o1>>11)+1)*2^-53, u2 = (o2>>11)*2^-53,
 * g = sqrt(-2 ln u1) cos(2 pi u2), and xi_p = g_p/||g_p||.  The first Q directions
 * do not depend on P.  EINVAL if d < 1, P < 1 or host_out is NULL. */
ksum_status ksum_generate_directions(int32_t d, int32_t P, uint64_t seed, double *host_out);

/* Workspace bytes an execution with N sources and M targets needs, without a
 * plan (host only).  EINVAL for invalid parameters or N, M < 1. */
ksum_status ksum_workspace_bytes(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params,
                                 int64_t N, int64_t M, size_t *bytes);

/* Create a plan for dimension d >= 1 and P >= 1 directions (the problem statement
 * of Sec. 1 fixes d, the kernel and its parameters; Sec. 2.3 the directions).
 * params may be NULL (defaults).  Draws the directions, precomputes the window
 * and coefficient tables and uploads them to params->device.  The plan owns
 * everything it allocates; release it with ksum_plan_destroy.
 * EINVAL / EUNSUPPORTED for bad arguments, ENOMEM, EDEVICE without a device. */
ksum_status ksum_plan_create(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params,
                             ksum_plan **out);

/* Release a plan (NULL is accepted).  Its tables are freed in the order of the
 * library's own stream after the plan's work on every stream it ran on (the host
 * does not wait); if its work was captured into a graph, or ran on more streams
 * than the plan tracks, the call first synchronises the plan's device.  A graph
 * holding the plan's work must not be launched after the plan is released. */
ksum_status ksum_plan_destroy(ksum_plan *plan);

/* Copy the plan's directions (P*d FP64, row-major) to host_out. */
ksum_status ksum_get_directions(const ksum_plan *plan, double *host_out);

/* Workspace bytes ksum_execute needs for N sources and M targets. */
ksum_status ksum_workspace_size(const ksum_plan *plan, int64_t N, int64_t M, size_t *bytes);

/* Forward sliced kernel sum (Algorithm "Sliced Fast Fourier Summation").
 *   x   device float[N][d] sources          y  device float[M][d] targets
 *   w   device float[N] weights             s  device float[M] output (overwritten)
 *   ws  device workspace of ws_bytes >= ksum_workspace_size(plan, N, M)
 *   stream  hipStream_t (as void*) the work is enqueued on
 * x and y may alias; s must not overlap any input or the workspace.  Without the
 * opt-in input check the call only enqueues kernels on the stream (no copies, no
 * memsets, no host synchronisation), so it may be captured into a HIP graph; a
 * launch of the graph reads and writes the buffers the capture saw.
 * EINVAL for null pointers or N, M < 1; EWORKSPACE if ws_bytes is too small. */
ksum_status ksum_execute(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M,
                         const float *w, float *s, void *ws, size_t ws_bytes, void *stream);

/* As ksum_execute with FP64 inputs x, y, w (converted to FP32 as they are read). */
ksum_status ksum_execute_f64in(ksum_plan *plan, const double *x, int64_t N, const double *y, int64_t M,
                               const double *w, float *s, void *ws, size_t ws_bytes, void *stream);

/* As ksum_execute, and also writes the intermediate arrays probe names (probe may
 * be NULL).  Requesting perm makes ties in the sort ordered by union index. */
ksum_status ksum_execute_probe(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M,
                               const float *w, float *s, void *ws, size_t ws_bytes, void *stream,
                               const ksum_probe *probe);

/* As ksum_execute_probe with FP64 inputs x, y, w (converted to FP32 as they are read;
 * the probed z are the FP32 projections of the converted inputs). */
ksum_status ksum_execute_probe_f64in(ksum_plan *plan, const double *x, int64_t N, const double *y, int64_t M,
                                     const double *w, float *s, void *ws, size_t ws_bytes, void *stream,
                                     const ksum_probe *probe);

/* Forward sum for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) and so cannot
 * provide the workspace of ksum_execute.  Same arguments and result as
 * ksum_execute without ws / ws_bytes: the workspace is a static device array of
 * KSUM_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from the first
 * use on that GPU until the process ends.  The slices run in batches of the
 * plan's batch size or fewer, as many as fit the array; the result does not depend
 * on the batch size.  Allocates nothing (no hipMalloc, hipFree or allocating
 * library call).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads, other plans) race and must be
 * ordered by the caller; each call writes every part of the array it reads before
 * reading it.  EWORKSPACE if one slice of N sources and M targets needs more than
 * the array holds; other errors as for ksum_execute. */
#define KSUM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ksum_status ksum_execute_noalloc(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M,
                                 const float *w, float *s, void *stream);

/* Workspace bytes ksum_backward needs for N sources and M targets. */
ksum_status ksum_backward_workspace_size(const ksum_plan *plan, int64_t N, int64_t M, size_t *bytes);

/* Gradients of a loss L through the forward sum s = ksum_execute(plan, x, y, w), given
 * grad_s = dL/ds (device float[M]).  With the directions held fixed, the chain rule
 * through the projections of Algorithm "Sliced Fast Fourier Summation" gives
 *   grad_w[n]    = (1/P) sum_p sum_m grad_s[m] k(<xi_p,x_n>, <xi_p,y_m>)   (the forward sum with
 *                  sources y weighted by grad_s and targets x)
 *   grad_y[m][.] = grad_s[m]/P sum_p D^y[m][p] xi_p,  D^y[m][p] = d/dz sum_n w_n f(|<xi_p,x_n> - z|) at
 *                  z = <xi_p,y_m>
 *   grad_x[n][.] = w[n]/P sum_p D^x[n][p] xi_p,       D^x[n][p] = d/dz sum_m grad_s[m] f(|<xi_p,y_m> - z|)
 *                  at z = <xi_p,x_n>
 * The derivative sums come from the same 1-D methods as the forward sums: Fourier
 * summation (Sec. 3.1) with the coefficients c_k times 2 pi i k, and the sorted
 * prefix sums of Sec. 3.2 with sign(0) = 0 (a source at the target's position adds
 * nothing); the rescaling bounds and tau are held constant.
 *   x, y, w       the forward inputs (device float, layouts as in ksum_execute)
 *   grad_s        device float[M]
 *   grad_x        device float[N][d] output, or NULL to skip
 *   grad_y        device float[M][d] output, or NULL to skip
 *   grad_w        device float[N] output, or NULL to skip
 *   ws            device workspace of ws_bytes >= ksum_backward_workspace_size(plan, N, M)
 * Outputs are overwritten; none may overlap an input or the workspace.  Errors as
 * for ksum_execute. */
ksum_status ksum_backward(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M, const float *w,
                          const float *grad_s, float *grad_x, float *grad_y, float *grad_w, void *ws,
                          size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Request server (continuous batching on one GPU).  A request is one forward sum
 * (ksum_execute) and, when grad_s is not NULL, its backward (ksum_backward), with
 * the plan given by (d, P, kernel, params).  ksum_server_submit queues it; a worker
 * thread of the server starts queued requests in arrival order as soon as one of
 * `slots` HIP streams is free and the request's workspace fits the server's HBM
 * arena of `hbm_bytes` (admission by footprint; a request that does not fit lets
 * later ones pass at most 16 times).  Requests run concurrently on their streams;
 * plans are created once per distinct key and kept with their device tables.  All
 * kernels are deterministic, so a result is bitwise the same alone and in the mix.
 * Device pointers in a request are the caller's and must stay valid until the
 * request's completion has been returned by ksum_server_poll.
 * ------------------------------------------------------------------------- */
typedef struct ksum_server ksum_server;

typedef struct {
  uint64_t tag;              /* caller's identifier, returned in the completion */
  int32_t d, P;
  ksum_kernel kernel;
  ksum_params params;        /* params.directions and params.device are ignored */
  const float *x;            /* device float[N][d] sources */
  int64_t N;
  const float *y;            /* device float[M][d] targets */
  int64_t M;
  const float *w;            /* device float[N] weights */
  float *s;                  /* device float[M] output */
  const float *grad_s;       /* device float[M] upstream gradient, or NULL for no backward */
  float *grad_x, *grad_y, *grad_w;   /* backward outputs (each may be NULL) */
  void *ready_event;         /* hipEvent_t recorded after the work that writes x, y, w, grad_s; the
                                request's kernels wait for it.  NULL: the inputs must be complete on
                                the device when ksum_server_submit is called.  The event must not be
                                recorded again or destroyed before the request's completion is polled */
} ksum_request;

typedef struct {
  uint64_t tag;
  int32_t status;            /* ksum_status of the request */
  double t_submit, t_start, t_end;   /* host steady-clock seconds: queued, started, seen complete */
  size_t ws_bytes;           /* workspace the request held */
} ksum_completion;

typedef struct {
  int64_t submitted, finished, queued, running, plans;
  size_t arena_bytes, arena_used, arena_peak;
} ksum_server_info;

/* Create a server on `device` with `slots` streams (1..64) and an HBM arena of
 * hbm_bytes (allocated once here).  EINVAL, ENOMEM, EDEVICE. */
ksum_status ksum_server_create(int32_t device, int32_t slots, size_t hbm_bytes, ksum_server **out);
/* Queue a request (copied; host call, returns at once).  EINVAL for missing
 * pointers or bad sizes, the status of ksum_check_params for bad plan parameters. */
ksum_status ksum_server_submit(ksum_server *server, const ksum_request *request);
/* Move up to max_out finished requests into out (host array); *n_out = count. */
ksum_status ksum_server_poll(ksum_server *server, ksum_completion *out, int32_t max_out, int32_t *n_out);
/* Block until no request is queued or running. */
ksum_status ksum_server_drain(ksum_server *server);
/* Counters of the server (host). */
ksum_status ksum_server_stats(ksum_server *server, ksum_server_info *info);
/* Finish every queued request, then release the streams, plans and arena. */
ksum_status ksum_server_destroy(ksum_server *server);

/* Per-kernel timing (diagnostic).  While enabled, ksum_execute records HIP events
 * on its stream around every kernel it launches (a few microseconds of overhead
 * per kernel); ksum_stage_times synchronises with the last event and returns,
 * for each stage, the accumulated milliseconds and the number of launches since
 * timing was enabled.  The plan holds 16384 events between two reads: launches
 * beyond them are not timed, and the next ksum_stage_times still fills its outputs
 * but returns KSUM_EWORKSPACE.  Not thread-safe: time one execution stream at a time.
 * Stages are numbered 0..ksum_stage_count()-1 and named by ksum_stage_name(). */
ksum_status ksum_set_timing(ksum_plan *plan, int32_t enable);
ksum_status ksum_stage_times(ksum_plan *plan, double *ms_out, int64_t *calls_out);
int32_t ksum_stage_count(void);
const char *ksum_stage_name(int32_t stage);

#ifdef __cplusplus
}
#endif

#endif /* KSUM_H */
