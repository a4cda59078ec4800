// C ABI of the ksum library: parameter handling, plans, workspace layout and
// the execution schedule (one dependency chain per slice batch on the caller's
// stream; no host synchronisation inside ksum_execute).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "internal.h"

namespace ksum {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int window_degree_for(int m);
int nfft_share_for(int W);
hipError_t launch_bounds_probe(const ExecArgs &a, double *bounds_out);

static ksum_status fail(ksum_status st, const std::string &msg) {
  set_error(msg);
  return st;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// bfloat16 of a finite float, round to nearest even, and back
static uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static float bf16_to_float(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Resolved method of a kernel: the smooth part's transform for the Fourier
// kernels, SORT for the negative distance.
static int resolve_method(ksum_kernel kernel, const ksum_params &p) {
  if (kernel == KSUM_NEGDIST) return KSUM_1D_SORT;
  if (p.method != KSUM_1D_AUTO) return p.method;
  if (kernel == KSUM_GAUSSIAN) return p.n_coeff <= 64 ? KSUM_1D_NDFT : KSUM_1D_NFFT;
  return KSUM_1D_NFFT;
}

static double resolve_T(ksum_kernel kernel, int method, double T) {
  if (T > 0.0) return T;
  if (kernel == KSUM_GAUSSIAN) return method == KSUM_1D_NDFT ? 0.045 : 0.02;
  if (kernel == KSUM_LAPLACIAN || kernel == KSUM_MATERN) return 0.125;
  return 0.0;
}

// NFFT window cells for grid n, threshold T, half-width m (one cell of margin on
// each side of the base-cell range [floor(-nT), floor(nT)]).
static void nfft_window(int n, double T, int m, int *lo, int *cells) {
  const int i0lo = (int)std::floor(-(double)n * T) - 1;
  const int i0hi = (int)std::floor((double)n * T) + 1;
  *lo = i0lo - m + 1;
  *cells = (i0hi + m) - *lo + 1;
}

static ksum_status validate(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params &p) {
  if (d < 1 || d > (1 << 20)) return fail(KSUM_EINVAL, "d must be in [1, 2^20]");
  if (P < 1 || P > (1 << 24)) return fail(KSUM_EINVAL, "P must be in [1, 2^24]");
  if (kernel != KSUM_GAUSSIAN && kernel != KSUM_LAPLACIAN && kernel != KSUM_NEGDIST && kernel != KSUM_MATERN)
    return fail(KSUM_EINVAL, "unknown kernel");
  if (p.method < KSUM_1D_AUTO || p.method > KSUM_1D_SORT) return fail(KSUM_EINVAL, "unknown method");
  if (p.precision != KSUM_FP32 && p.precision != KSUM_SPLIT_BF16)
    return fail(KSUM_EINVAL, "unknown precision");
  if (p.slice_batch < 0) return fail(KSUM_EINVAL, "slice_batch must be >= 0");
  if (p.device < 0) return fail(KSUM_EINVAL, "device must be >= 0");
  if (p.check_finite != 0 && p.check_finite != 1) return fail(KSUM_EINVAL, "check_finite must be 0 or 1");
  if (kernel == KSUM_NEGDIST) {
    if (p.method != KSUM_1D_AUTO && p.method != KSUM_1D_SORT)
      return fail(KSUM_EUNSUPPORTED, "the negative distance kernel uses the sort method");
    return KSUM_OK;
  }
  if (!(p.sigma > 0.0) || !std::isfinite(p.sigma)) return fail(KSUM_EINVAL, "sigma must be finite and > 0");
  if (p.n_coeff < 2 || p.n_coeff > 4096 || (p.n_coeff & 1))
    return fail(KSUM_EINVAL, "n_coeff must be even and in [2, 4096]");
  if (!(p.coeff_eps >= 0.0)) return fail(KSUM_EINVAL, "coeff_eps must be >= 0");
  if (!(p.T >= 0.0 && p.T < 0.25)) return fail(KSUM_EINVAL, "T must satisfy 0 < T < 0.25 (0 = default)");
  if (p.method == KSUM_1D_SORT) return fail(KSUM_EUNSUPPORTED, "this kernel has no pure sort method");
  const int method = resolve_method(kernel, p);
  if (method == KSUM_1D_NFFT) {
    if (p.oversample < 2 || p.oversample > 8) return fail(KSUM_EINVAL, "oversample must be in [2, 8]");
    if (p.window_m < 2 || p.window_m > 8) return fail(KSUM_EINVAL, "window_m must be in [2, 8]");
    const int64_t n = (int64_t)p.oversample * p.n_coeff;
    if (n > 8192 || (n & (n - 1))) return fail(KSUM_EUNSUPPORTED, "NFFT grid must be a power of two <= 8192");
    int lo, cells;
    nfft_window((int)n, resolve_T(kernel, method, p.T), p.window_m, &lo, &cells);
    if (cells > n) return fail(KSUM_EUNSUPPORTED, "NFFT window wider than the grid (T too large)");
    if (nfft_share_for(cells) == 0) return fail(KSUM_EUNSUPPORTED, "NFFT window does not fit LDS");
  }
  return KSUM_OK;
}

Layout make_layout(const ksum_plan &pl, int64_t N, int64_t M, int32_t batch, bool allow_presplit) {
  Layout y;
  y.N = N;
  y.M = M;
  y.L = N + M;
  y.B = pl.params.slice_batch > 0 ? std::min(pl.params.slice_batch, pl.P) : pl.P;
  y.B = std::min(y.B, kMaxBatch);
  if (batch > 0) y.B = std::min(y.B, batch);
  const int64_t B = y.B;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  y.off_misc = take(8 * sizeof(double));
  y.off_wpart = take(kWsumBlocks * sizeof(double));
  y.off_params = take(B * sizeof(SliceParams));
  y.off_bounds = take(B * 2 * sizeof(uint32_t));
  y.off_counter = take(64);
  y.off_bounds_part = take((size_t)256 * kGemmBlocksPerCU * B * 2 * sizeof(uint32_t));
  y.off_z = take((size_t)B * y.L * sizeof(float));
  // per-slice sums that pass through HBM: NDFT output and the negative-distance sort
  // output (t1), the Laplacian's sorted part (t2); the NFFT interpolation adds its
  // part directly into the slice average
  const bool need_t1 = (pl.kernel == KSUM_NEGDIST) || (pl.use_fourier && pl.method == KSUM_1D_NDFT);
  y.off_t1 = need_t1 ? take((size_t)B * M * sizeof(float)) : 0;
  y.off_t2 = (pl.kernel == KSUM_LAPLACIAN) ? take((size_t)B * M * sizeof(float)) : y.off_t1;
  y.off_sacc = take((size_t)M * sizeof(double));
  y.off_wf = take((size_t)N * sizeof(float));
  if (pl.use_fourier) {
    y.off_coef = take((size_t)B * (pl.K + 1) * sizeof(float));
    if (pl.method == KSUM_1D_NDFT) {
      y.ndft_chunks = (int32_t)((N + 4095) / 4096);
      y.off_fpart = take((size_t)B * y.ndft_chunks * (pl.K + 1) * sizeof(float2));
    } else {
      nfft_window(pl.n_grid, pl.params.T, pl.params.window_m, &y.win_lo, &y.win_cells);
      y.nfft_chunks = (int32_t)((N + (int64_t)256 * kNfftPPL - 1) / ((int64_t)256 * kNfftPPL));
      y.off_fpart = take((size_t)B * y.nfft_chunks * y.win_cells * sizeof(float));
      y.off_grid = take((size_t)B * y.win_cells * sizeof(float));
    }
    if (pl.lap_L > 0) y.off_lapv = take((size_t)B * pl.lap_L * sizeof(double));
  }
  if (pl.use_sort) {
    const int64_t L = y.L;
    y.nb = (int32_t)std::min<int64_t>(2048, std::max<int64_t>(64, next_pow2((L + 511) / 512)));
    y.sort_groups = (int32_t)((L + kSortHalf - 1) / kSortHalf + 1);
    // chunks of about two of the scatter's largest tiles, so that its tiles are full
    y.sort_nch = (int32_t)std::min<int64_t>(kSortChunkMax, std::max<int64_t>(1, (L + kSortChunkLen - 1) / kSortChunkLen));
    y.sort_chunk = (L + y.sort_nch - 1) / y.sort_nch;
    y.off_hcnt = take((size_t)B * y.sort_nch * y.nb * sizeof(uint32_t));
    y.off_hsum = take((size_t)B * y.sort_nch * y.nb * 2 * sizeof(long long));
    y.off_bpre = take((size_t)B * y.nb * 2 * sizeof(long long));
    y.off_boff = take((size_t)B * (y.nb + 1) * sizeof(uint32_t));
    y.off_tot = take((size_t)B * 2 * sizeof(long long));
    y.off_keys = take((size_t)B * L * sizeof(unsigned long long));
    y.off_keys2 = take((size_t)B * L * sizeof(unsigned long long));
    y.off_desc = take((size_t)B * y.sort_groups * sizeof(int4));
    y.off_fail = take((64 + (size_t)B * y.sort_groups) * sizeof(uint32_t));
  }
  y.off_flag = take(64);
  // split-BF16 plans with many slice tiles split the points once per call instead of
  // once per tile and batch
  y.presplit = allow_presplit && split_tiled(pl);
  if (y.presplit) {
    y.split_rows = (int64_t)align_up((size_t)y.L, 2 * kGemmBM);
    y.off_split = take((size_t)y.split_rows * pl.d_pad * 2 * sizeof(uint16_t));
  }
  y.total = o;
  return y;
}

static void fill_defaults(ksum_kernel kernel, ksum_params *p) {
  std::memset(p, 0, sizeof(*p));
  p->sigma = 1.0;
  p->seed = 0;
  p->directions = nullptr;
  p->n_coeff = (kernel == KSUM_LAPLACIAN) ? 256 : (kernel == KSUM_MATERN) ? 1024 : 64;
  p->coeff_eps = 0.0;
  p->T = 0.0;
  p->oversample = 2;
  p->window_m = 6;
  p->method = KSUM_1D_AUTO;
  p->precision = KSUM_FP32;
  p->slice_batch = 0;
  p->device = 0;
  p->check_finite = 0;
}

static void free_timer(ksum_plan *pl) {
  if (!pl->timer) return;
  for (hipEvent_t e : pl->timer->ev) (void)hipEventDestroy(e);
  delete pl->timer;
  pl->timer = nullptr;
}

// The library's own stream on a device (non-blocking, default priority), made at the
// first use: plan tables are allocated, uploaded and freed in its order, so that
// releasing a plan waits for the plan's own work and not for the whole device.
static std::mutex g_stream_mu;
static hipStream_t g_lib_stream[64] = {};

static hipStream_t library_stream(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_stream_mu);
  if (!g_lib_stream[dev] && hipStreamCreateWithFlags(&g_lib_stream[dev], hipStreamNonBlocking) != hipSuccess)
    g_lib_stream[dev] = nullptr;
  return g_lib_stream[dev];
}

// Device copy of a host table, allocated from the device's stream-ordered pool.
static hipError_t upload(hipStream_t ls, void **dst, const void *src, size_t bytes) {
  hipError_t e = hipMallocAsync(dst, bytes, ls);
  if (e == hipSuccess) e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, ls);
  if (e == hipSuccess) e = hipStreamSynchronize(ls);
  return e;
}

// Records that the plan's work was enqueued on `stream` (after every call that launches).
static void note_use(ksum_plan *pl, hipStream_t stream) {
  std::lock_guard<std::mutex> lock(pl->use_mu);
  // work captured into a graph runs whenever the graph is launched, which no event
  // recorded now can follow: the plan's release then waits for the whole device
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
    pl->use_overflow = true;
    return;
  }
  int i = 0;
  while (i < pl->n_use && pl->use_stream[i] != stream) ++i;
  if (i == pl->n_use) {
    if (pl->n_use == ksum_plan::kUseSlots ||
        hipEventCreateWithFlags(&pl->use_event[i], hipEventDisableTiming) != hipSuccess) {
      pl->use_overflow = true;
      return;
    }
    pl->use_stream[i] = stream;
    ++pl->n_use;
  }
  if (hipEventRecord(pl->use_event[i], stream) != hipSuccess) pl->use_overflow = true;
}

// Releases a plan's tables in the library stream's order after the plan's own work
// (the device must be current).
static void free_plan(ksum_plan *pl) {
  if (!pl) return;
  free_timer(pl);
  void *tabs[] = {pl->d_dirs, pl->d_dirs_hi, pl->d_dirs_lo, pl->d_dirs_tiled, pl->d_dirsT, pl->d_deconv, pl->d_twiddle,
                  pl->d_costab};
  bool on_device = pl->n_use > 0;
  for (void *t : tabs) on_device |= t != nullptr;
  if (!on_device) {
    delete pl;
    return;
  }
  hipStream_t ls = library_stream(pl->params.device);
  if (pl->use_overflow || !ls) (void)hipDeviceSynchronize();
  for (int i = 0; i < pl->n_use; ++i) {
    if (ls) (void)hipStreamWaitEvent(ls, pl->use_event[i], 0);
    (void)hipEventDestroy(pl->use_event[i]);
  }
  for (void *t : tabs) {
    if (!t) continue;
    if (ls) (void)hipFreeAsync(t, ls);
    else (void)hipFree(t);
  }
  delete pl;
}

}  // namespace ksum

using namespace ksum;

extern "C" {

const char *ksum_version(void) { return "ksum 0.1.0 (gfx950)"; }

const char *ksum_status_string(ksum_status st) {
  switch (st) {
    case KSUM_OK: return "KSUM_OK";
    case KSUM_EINVAL: return "KSUM_EINVAL";
    case KSUM_EUNSUPPORTED: return "KSUM_EUNSUPPORTED";
    case KSUM_ENOMEM: return "KSUM_ENOMEM";
    case KSUM_EWORKSPACE: return "KSUM_EWORKSPACE";
    case KSUM_ENONFINITE: return "KSUM_ENONFINITE";
    case KSUM_EDEVICE: return "KSUM_EDEVICE";
  }
  return "KSUM_UNKNOWN";
}

const char *ksum_last_error(void) { return g_last_error.c_str(); }

ksum_status ksum_params_default(ksum_kernel kernel, ksum_params *out) {
  if (!out) return fail(KSUM_EINVAL, "out is NULL");
  if (kernel != KSUM_GAUSSIAN && kernel != KSUM_LAPLACIAN && kernel != KSUM_NEGDIST && kernel != KSUM_MATERN)
    return fail(KSUM_EINVAL, "unknown kernel");
  fill_defaults(kernel, out);
  return KSUM_OK;
}

ksum_status ksum_check_params(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params) {
  ksum_params p;
  if (params) p = *params; else fill_defaults(kernel, &p);
  return validate(d, P, kernel, p);
}

ksum_status ksum_generate_directions(int32_t d, int32_t P, uint64_t seed, double *host_out) {
  if (d < 1 || P < 1) return fail(KSUM_EINVAL, "d and P must be >= 1");
  if (!host_out) return fail(KSUM_EINVAL, "host_out is NULL");
  generate_directions(d, P, seed, host_out);
  return KSUM_OK;
}

// Fills the host-side fields of a plan (no device access).
static ksum_status plan_host_setup(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params,
                                   ksum_plan *pl) {
  ksum_params p;
  if (params) p = *params; else fill_defaults(kernel, &p);
  const ksum_status st = validate(d, P, kernel, p);
  if (st != KSUM_OK) return st;
  pl->d = d;
  pl->P = P;
  pl->kernel = kernel;
  pl->method = resolve_method(kernel, p);
  p.T = resolve_T(kernel, pl->method, p.T);
  pl->params = p;
  pl->params.directions = nullptr;
  pl->use_sort = (kernel == KSUM_NEGDIST || kernel == KSUM_LAPLACIAN);
  pl->use_fourier = (kernel != KSUM_NEGDIST);
  // the split-BF16 GEMM takes K steps of 2 kGemmBK
  const int kstep = (p.precision == KSUM_SPLIT_BF16) ? 2 * kGemmBK : kGemmBK;
  pl->d_pad = (int32_t)((d + kstep - 1) / kstep * kstep);
  // padding rows of zeros: a GEMM tile of up to 2 kGemmBM slices may start at any slice below P
  pl->P_pad = (int32_t)((P + kGemmBM - 1) / kGemmBM * kGemmBM + 2 * kGemmBM);
  pl->Pk = (int32_t)((P + kGemmBK - 1) / kGemmBK * kGemmBK);
  pl->cd = std::sqrt(M_PI) * std::exp(std::lgamma((d + 1) / 2.0) - std::lgamma(d / 2.0));
  pl->sort_const = (kernel == KSUM_LAPLACIAN) ? pl->cd / p.sigma : pl->cd;
  pl->gauss_logc = std::log((double)d * M_PI / std::sqrt(2.0)) - std::lgamma((d + 2) / 2.0);
  pl->matern_c3 = std::sqrt(3.0 * M_PI) * std::exp(std::lgamma(d / 2.0 + 1.5) - std::lgamma(d / 2.0));
  if (pl->use_fourier) {
    pl->K = (pl->method == KSUM_1D_NDFT) ? p.n_coeff / 2 : p.n_coeff / 2 - 1;
    if (pl->method == KSUM_1D_NFFT) pl->n_grid = p.oversample * p.n_coeff;
    if (kernel == KSUM_LAPLACIAN || kernel == KSUM_MATERN) pl->lap_L = 16 * p.n_coeff;
  }
  pl->dirs.resize((size_t)P * d);
  if (params && params->directions) {
    std::memcpy(pl->dirs.data(), params->directions, sizeof(double) * (size_t)P * d);
  } else {
    generate_directions(d, P, p.seed, pl->dirs.data());
  }
  if (pl->method == KSUM_1D_NFFT) {
    std::string err;
    if (!build_window_poly(p.window_m, pl->n_grid, p.oversample, &pl->poly, &err))
      return fail(KSUM_EUNSUPPORTED, err);
  }
  return KSUM_OK;
}

ksum_status ksum_workspace_bytes(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params,
                                 int64_t N, int64_t M, size_t *bytes) {
  if (!bytes) return fail(KSUM_EINVAL, "bytes is NULL");
  if (N < 1 || M < 1) return fail(KSUM_EINVAL, "N and M must be >= 1");
  if (N + M > 0x7fffffffLL) return fail(KSUM_EUNSUPPORTED, "N + M must be < 2^31");
  ksum_plan tmp;
  ksum_params p;
  if (params) p = *params; else fill_defaults(kernel, &p);
  p.directions = nullptr;   // the directions do not change the size
  const ksum_status st = plan_host_setup(d, P, kernel, &p, &tmp);
  if (st != KSUM_OK) return st;
  *bytes = make_layout(tmp, N, M).total;
  return KSUM_OK;
}

ksum_status ksum_plan_create(int32_t d, int32_t P, ksum_kernel kernel, const ksum_params *params,
                             ksum_plan **out) {
  if (!out) return fail(KSUM_EINVAL, "out is NULL");
  *out = nullptr;
  ksum_plan *pl = new (std::nothrow) ksum_plan();
  if (!pl) return fail(KSUM_ENOMEM, "host allocation failed");
  ksum_status st = plan_host_setup(d, P, kernel, params, pl);
  if (st != KSUM_OK) {
    free_plan(pl);
    return st;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= pl->params.device) {
    free_plan(pl);
    return fail(KSUM_EDEVICE, "no HIP device with the requested ordinal");
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(pl->params.device) != hipSuccess) {
    free_plan(pl);
    return fail(KSUM_EDEVICE, "hipSetDevice failed");
  }
  auto dev_fail = [&](ksum_status s, const char *what) {
    free_plan(pl);
    (void)hipSetDevice(prev);
    return fail(s, what);
  };
  hipStream_t ls = library_stream(pl->params.device);
  if (!ls) return dev_fail(KSUM_EDEVICE, "could not create the library stream");
  auto up = [&](auto **dst, const void *src, size_t bytes) {
    void *p = nullptr;
    const hipError_t e = upload(ls, &p, src, bytes);
    *dst = static_cast<std::remove_reference_t<decltype(**dst)> *>(p);
    return e == hipSuccess;
  };
  // directions, FP32, zero padded to [P_pad][d_pad]
  std::vector<float> hd((size_t)pl->P_pad * pl->d_pad, 0.f);
  for (int32_t p = 0; p < P; ++p)
    for (int32_t i = 0; i < d; ++i) hd[(size_t)p * pl->d_pad + i] = (float)pl->dirs[(size_t)p * d + i];
  if (!up(&pl->d_dirs, hd.data(), hd.size() * sizeof(float))) return dev_fail(KSUM_ENOMEM, "device allocation");
  {
    // transposed FP32 directions [d][Pk] for the back-projection of the backward pass
    std::vector<float> ht((size_t)d * pl->Pk, 0.f);
    for (int32_t p = 0; p < P; ++p)
      for (int32_t i = 0; i < d; ++i) ht[(size_t)i * pl->Pk + p] = (float)pl->dirs[(size_t)p * d + i];
    if (!up(&pl->d_dirsT, ht.data(), ht.size() * sizeof(float))) return dev_fail(KSUM_ENOMEM, "device allocation");
  }
  if (pl->params.precision == KSUM_SPLIT_BF16) {
    // hi = bf16(xi), lo = bf16(xi - hi) of the FP32 directions, round to nearest even
    std::vector<uint16_t> hh(hd.size()), hl(hd.size());
    for (size_t i = 0; i < hd.size(); ++i) {
      hh[i] = bf16_rne(hd[i]);
      hl[i] = bf16_rne(hd[i] - bf16_to_float(hh[i]));
    }
    const size_t nb = hd.size() * sizeof(uint16_t);
    if (!up(&pl->d_dirs_hi, hh.data(), nb) || !up(&pl->d_dirs_lo, hl.data(), nb))
      return dev_fail(KSUM_ENOMEM, "device allocation");
    if (split_tiled(*pl)) {
      // the same values step-tiled for the GEMM fed by direct LDS copies
      std::vector<uint16_t> ht(2 * hd.size());
      const int nst = pl->d_pad / kGemmBK;
      for (int s = 0; s < nst; ++s)
        for (int64_t r = 0; r < pl->P_pad; ++r) {
          uint16_t *dst = ht.data() + ((size_t)s * pl->P_pad + r) * 32;
          const size_t src = (size_t)r * pl->d_pad + (size_t)s * kGemmBK;
          for (int c = 0; c < 4; ++c) {
            const uint16_t *from = (c < 2 ? hh.data() : hl.data()) + src + (c & 1) * 8;
            std::copy(from, from + 8, dst + 8 * (c ^ tile_swz(r)));
          }
        }
      if (!up(&pl->d_dirs_tiled, ht.data(), 2 * nb)) return dev_fail(KSUM_ENOMEM, "device allocation");
    }
  }
  if (pl->method == KSUM_1D_NFFT) {
    const int n = pl->n_grid, m = pl->params.window_m, os = pl->params.oversample;
    // window normalised to phi(0) = 1 in the polynomials; deconvolution 1/(n phihat/phi0)^2
    const double b = M_PI * (2.0 - 1.0 / os);
    const double phi0 = std::sinh(b * m) / (M_PI * m);
    std::vector<float> dc(pl->K + 1);
    for (int k = 0; k <= pl->K; ++k) {
      const double ph = (double)n * kb_phihat(m, n, os, k) / phi0;
      dc[k] = (float)(1.0 / (ph * ph));
    }
    std::vector<float2> tw(n);
    for (int j = 0; j < n; ++j) {
      const double ang = -2.0 * M_PI * (double)j / (double)n;
      tw[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if (!up(&pl->d_deconv, dc.data(), dc.size() * sizeof(float)) ||
        !up(&pl->d_twiddle, tw.data(), tw.size() * sizeof(float2)))
      return dev_fail(KSUM_ENOMEM, "device allocation");
  }
  if (pl->lap_L > 0) {
    std::vector<double> ct(pl->lap_L);
    for (int j = 0; j < pl->lap_L; ++j) ct[j] = std::cos(2.0 * M_PI * (double)j / (double)pl->lap_L);
    if (!up(&pl->d_costab, ct.data(), ct.size() * sizeof(double))) return dev_fail(KSUM_ENOMEM, "device allocation");
  }
  (void)hipSetDevice(prev);
  *out = pl;
  return KSUM_OK;
}

ksum_status ksum_plan_destroy(ksum_plan *plan) {
  if (!plan) return KSUM_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(plan->params.device);
  free_plan(plan);
  (void)hipSetDevice(prev);
  return KSUM_OK;
}

ksum_status ksum_get_directions(const ksum_plan *plan, double *host_out) {
  if (!plan || !host_out) return fail(KSUM_EINVAL, "null argument");
  std::memcpy(host_out, plan->dirs.data(), sizeof(double) * plan->dirs.size());
  return KSUM_OK;
}

ksum_status ksum_workspace_size(const ksum_plan *plan, int64_t N, int64_t M, size_t *bytes) {
  if (!plan || !bytes) return fail(KSUM_EINVAL, "null argument");
  if (N < 1 || M < 1) return fail(KSUM_EINVAL, "N and M must be >= 1");
  if (N + M > 0x7fffffffLL) return fail(KSUM_EUNSUPPORTED, "N + M must be < 2^31");
  *bytes = make_layout(*plan, N, M).total;
  return KSUM_OK;
}

// One pass of the hot path over all slices, batch by batch, on the plan's device:
// forward sums into s, or (deriv) the per-target derivative sums into dout[M][ldd].
// Stages of one slice batch after the projection and the set-up: the 1-D sums and the
// running average into s or, in derivative mode, the per-slice derivative sums (a.dout).
static hipError_t post_projection(const ExecArgs &a, float *s) {
  const ksum_plan *plan = a.plan;
  hipError_t e = hipSuccess;
  if (plan->use_fourier) e = (plan->method == KSUM_1D_NDFT) ? launch_ndft(a) : launch_nfft(a);
  if (e == hipSuccess && plan->use_sort) e = launch_sort_path(a);
  const bool first = a.p0 == 0, last = a.p0 + a.nsl >= plan->P;
  const bool interp = plan->use_fourier && plan->method == KSUM_1D_NFFT;
  if (e == hipSuccess) {
    if (interp) e = launch_nfft_interp(a, s, first, last);
    else if (a.deriv) e = launch_deriv_gather(a);
    else e = launch_accumulate(a, s, first, last);
  }
  return e;
}

static hipError_t run_pipeline(ksum_plan *plan, const Layout &lay, const void *x, const void *y, const void *w,
                               bool f64, float *s, bool deriv, float *dout, int64_t ldd, char *ws,
                               hipStream_t stream, const ksum_probe *probe) {
  ExecArgs a{};
  a.plan = plan;
  a.lay = &lay;
  a.ws = ws;
  a.stream = stream;
  a.x = x;
  a.y = y;
  a.f64in = f64;
  a.want_perm = probe && probe->perm;
  a.perm_out = probe ? probe->perm : nullptr;
  a.t_out = probe ? probe->t : nullptr;
  a.deriv = deriv;
  a.dout = dout;
  a.ldd = ldd;
  a.w = f64 ? wsp<float>(a, lay.off_wf) : static_cast<const float *>(w);
  hipError_t e = launch_weight_prep(a, f64 ? static_cast<const double *>(w) : nullptr);
  if (e == hipSuccess && lay.presplit) e = launch_split_points(a);
  for (int32_t p0 = 0; p0 < plan->P && e == hipSuccess; p0 += lay.B) {
    a.p0 = p0;
    a.nsl = std::min(lay.B, plan->P - p0);
    e = launch_projection(a);
    if (e == hipSuccess) e = launch_slice_setup(a);
    if (e == hipSuccess && probe && probe->z)
      e = hipMemcpyAsync(probe->z + (int64_t)p0 * lay.L, a.ws + lay.off_z, (size_t)a.nsl * lay.L * sizeof(float),
                         hipMemcpyDeviceToDevice, a.stream);
    if (e == hipSuccess && probe && probe->bounds) e = launch_bounds_probe(a, probe->bounds);
    if (e == hipSuccess) e = post_projection(a, s);
  }
  mark(a, -1);
  return e;
}

// The opt-in input check (params.check_finite): one pass over each array on the execution
// stream, then a wait for the flag it leaves in the workspace.  Runs before any other
// kernel of the call, so a call refused with KSUM_ENONFINITE writes no output.
struct CheckedArray {
  const void *p;
  int64_t n;
  bool f64;
};

static ksum_status check_inputs(std::initializer_list<CheckedArray> arrays, char *ws, const Layout &lay,
                                hipStream_t stream) {
  uint32_t *flag = reinterpret_cast<uint32_t *>(ws + lay.off_flag);
  hipError_t e = launch_fill_zero(reinterpret_cast<float *>(flag), 1, stream);
  for (const CheckedArray &a : arrays)
    if (e == hipSuccess) e = launch_check_finite(a.p, a.n, a.f64, flag, stream);
  uint32_t seen = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&seen, flag, sizeof(seen), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(KSUM_EDEVICE, std::string("input check failed: ") + hipGetErrorString(e));
  if (seen) return fail(KSUM_ENONFINITE, "an input holds a NaN or an infinity");
  return KSUM_OK;
}

static ksum_status check_exec_args(ksum_plan *plan, const void *x, int64_t N, const void *y, int64_t M,
                                   const void *w, const void *ws) {
  if (!plan) return fail(KSUM_EINVAL, "plan is NULL");
  if (!x || !y || !w || !ws) return fail(KSUM_EINVAL, "null device pointer");
  if (N < 1 || M < 1) return fail(KSUM_EINVAL, "N and M must be >= 1");
  if (N + M > 0x7fffffffLL) return fail(KSUM_EUNSUPPORTED, "N + M must be < 2^31");
  if ((uintptr_t)ws % 256 != 0) return fail(KSUM_EINVAL, "workspace must be 256-byte aligned");
  return KSUM_OK;
}

static ksum_status execute_impl(ksum_plan *plan, const void *x, int64_t N, const void *y, int64_t M,
                                const void *w, bool f64, float *s, void *ws, size_t ws_bytes, void *stream,
                                const ksum_probe *probe) {
  const ksum_status st = check_exec_args(plan, x, N, y, M, w, ws);
  if (st != KSUM_OK) return st;
  if (!s) return fail(KSUM_EINVAL, "null device pointer");
  const Layout lay = make_layout(*plan, N, M);
  if (ws_bytes < lay.total) return fail(KSUM_EWORKSPACE, "workspace too small");
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != plan->params.device && hipSetDevice(plan->params.device) != hipSuccess)
    return fail(KSUM_EDEVICE, "hipSetDevice failed");
  ksum_status cst = KSUM_OK;
  if (plan->params.check_finite) {
    const int64_t d = plan->d;
    cst = check_inputs({{x, N * d, f64}, {y, M * d, f64}, {w, N, f64}}, static_cast<char *>(ws), lay,
                       static_cast<hipStream_t>(stream));
  }
  hipError_t e = hipSuccess;
  if (cst == KSUM_OK) {
    e = run_pipeline(plan, lay, x, y, w, f64, s, false, nullptr, 0, static_cast<char *>(ws),
                     static_cast<hipStream_t>(stream), probe);
    note_use(plan, static_cast<hipStream_t>(stream));
  }
  if (prev != plan->params.device) (void)hipSetDevice(prev);
  if (cst != KSUM_OK) return cst;
  if (e != hipSuccess) return fail(KSUM_EDEVICE, std::string("HIP launch failed: ") + hipGetErrorString(e));
  return KSUM_OK;
}

// Workspace of the backward pass: the larger of the two pipeline layouts (targets y
// and targets x), then the derivative sums D [max(N, M)][Pk].
// Backward workspace: the forward layout with sources x and targets y (for dL/dy), the
// one with the roles exchanged (for dL/dw and dL/dx), and the derivative sums
// D^y [M][Pk] and D^x [N][Pk].
struct BackwardOffsets {
  size_t lx, dy, dx, total;
};

static BackwardOffsets backward_offsets(const ksum_plan &pl, int64_t N, int64_t M) {
  BackwardOffsets o;
  o.lx = align_up(make_layout(pl, N, M).total, 256);
  o.dy = align_up(o.lx + make_layout(pl, M, N).total, 256);
  o.dx = align_up(o.dy + (size_t)M * pl.Pk * sizeof(float), 256);
  o.total = o.dx + (size_t)N * pl.Pk * sizeof(float);
  return o;
}

ksum_status ksum_execute(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M, const float *w,
                         float *s, void *ws, size_t ws_bytes, void *stream) {
  return execute_impl(plan, x, N, y, M, w, false, s, ws, ws_bytes, stream, nullptr);
}

ksum_status ksum_execute_f64in(ksum_plan *plan, const double *x, int64_t N, const double *y, int64_t M,
                               const double *w, float *s, void *ws, size_t ws_bytes, void *stream) {
  return execute_impl(plan, x, N, y, M, w, true, s, ws, ws_bytes, stream, nullptr);
}

ksum_status ksum_execute_probe(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M,
                               const float *w, float *s, void *ws, size_t ws_bytes, void *stream,
                               const ksum_probe *probe) {
  return execute_impl(plan, x, N, y, M, w, false, s, ws, ws_bytes, stream, probe);
}

ksum_status ksum_execute_probe_f64in(ksum_plan *plan, const double *x, int64_t N, const double *y, int64_t M,
                                     const double *w, float *s, void *ws, size_t ws_bytes, void *stream,
                                     const ksum_probe *probe) {
  return execute_impl(plan, x, N, y, M, w, true, s, ws, ws_bytes, stream, probe);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Static scratch of ksum_execute_noalloc.  Every device the library runs on holds
// its own copy of this array (part of the code object loaded there) until the
// process ends.  Host code never passes the array's name to a kernel: the name is
// a host-side stand-in, and the device address of a device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[KSUM_NOALLOC_SCRATCH_BYTES];

namespace ksum {

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the scratch array on `dev`, which must be the current device.
static ksum_status scratch_address(int dev, char **out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(KSUM_EUNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KSUM_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return KSUM_OK;
}

}  // namespace ksum

extern "C" {

ksum_status ksum_execute_noalloc(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M,
                                 const float *w, float *s, void *stream) {
  if (!plan) return fail(KSUM_EINVAL, "plan is NULL");
  if (!x || !y || !w || !s) return fail(KSUM_EINVAL, "null device pointer");
  if (N < 1 || M < 1) return fail(KSUM_EINVAL, "N and M must be >= 1");
  if (N + M > 0x7fffffffLL) return fail(KSUM_EUNSUPPORTED, "N + M must be < 2^31");
  // the largest slice batch (at most the plan's) whose workspace fits the scratch; the
  // result does not depend on the batch size
  const size_t cap = KSUM_NOALLOC_SCRATCH_BYTES;
  const Layout one = make_layout(*plan, N, M, 1, false);
  if (one.total > cap)
    return fail(KSUM_EWORKSPACE, "N + M too large for the static scratch: one slice per batch needs " +
                                     std::to_string(one.total) + " bytes, the scratch holds " + std::to_string(cap));
  int32_t lo = 1, hi = make_layout(*plan, N, M).B;
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo + 1) / 2;
    if (make_layout(*plan, N, M, mid, false).total <= cap) lo = mid;
    else hi = mid - 1;
  }
  const Layout lay = make_layout(*plan, N, M, lo, false);
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != plan->params.device && hipSetDevice(plan->params.device) != hipSuccess)
    return fail(KSUM_EDEVICE, "hipSetDevice failed");
  char *ws = nullptr;
  ksum_status st = scratch_address(plan->params.device, &ws);
  if (st == KSUM_OK && plan->params.check_finite) {
    const int64_t d = plan->d;
    st = check_inputs({{x, N * d, false}, {y, M * d, false}, {w, N, false}}, ws, lay,
                      static_cast<hipStream_t>(stream));
  }
  if (st == KSUM_OK) {
    const hipError_t e = run_pipeline(plan, lay, x, y, w, false, s, false, nullptr, 0, ws,
                                      static_cast<hipStream_t>(stream), nullptr);
    note_use(plan, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) st = fail(KSUM_EDEVICE, std::string("HIP launch failed: ") + hipGetErrorString(e));
  }
  if (prev != plan->params.device) (void)hipSetDevice(prev);
  return st;
}

ksum_status ksum_backward_workspace_size(const ksum_plan *plan, int64_t N, int64_t M, size_t *bytes) {
  if (!plan || !bytes) return fail(KSUM_EINVAL, "null argument");
  if (N < 1 || M < 1) return fail(KSUM_EINVAL, "N and M must be >= 1");
  if (N + M > 0x7fffffffLL) return fail(KSUM_EUNSUPPORTED, "N + M must be < 2^31");
  *bytes = backward_offsets(*plan, N, M).total;
  return KSUM_OK;
}

ksum_status ksum_backward(ksum_plan *plan, const float *x, int64_t N, const float *y, int64_t M, const float *w,
                          const float *grad_s, float *grad_x, float *grad_y, float *grad_w, void *ws,
                          size_t ws_bytes, void *stream) {
  const ksum_status st = check_exec_args(plan, x, N, y, M, w, ws);
  if (st != KSUM_OK) return st;
  if (!grad_s) return fail(KSUM_EINVAL, "grad_s is NULL");
  const BackwardOffsets bo = backward_offsets(*plan, N, M);
  if (ws_bytes < bo.total) return fail(KSUM_EWORKSPACE, "workspace too small");
  if (!grad_x && !grad_y && !grad_w) return KSUM_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != plan->params.device && hipSetDevice(plan->params.device) != hipSuccess)
    return fail(KSUM_EDEVICE, "hipSetDevice failed");
  char *wsc = static_cast<char *>(ws);
  const hipStream_t sm = static_cast<hipStream_t>(stream);
  if (plan->params.check_finite) {
    const int64_t d = plan->d;
    const ksum_status cst = check_inputs({{x, N * d, false}, {y, M * d, false}, {w, N, false}, {grad_s, M, false}},
                                         wsc, make_layout(*plan, N, M), sm);
    if (cst != KSUM_OK) {
      if (prev != plan->params.device) (void)hipSetDevice(prev);
      return cst;
    }
  }
  const int64_t ldd = plan->Pk;
  const double invP = 1.0 / (double)plan->P;
  float *Dy = reinterpret_cast<float *>(wsc + bo.dy);
  float *Dx = reinterpret_cast<float *>(wsc + bo.dx);
  // The three sums share their projections.  dL/dy needs the sums with sources x and
  // targets y, whose union is (y, x); dL/dw (the sum with sources y, weights grad_s, and
  // targets x) and dL/dx (its derivative sums) share the union (x, y).  Both unions hold
  // the same points, so per slice batch the GEMM runs once: the second layout's Z is the
  // same matrix with its two column blocks exchanged, and its per-block min / max
  // partials are the same (the set-up of each layout then derives identical slice
  // parameters).  dL/dy_m = grad_s_m / P sum_p D^y[m][p] xi_p and
  // dL/dx_n = w_n / P sum_p D^x[n][p] xi_p follow by back-projection.
  const Layout ly = make_layout(*plan, N, M), lx = make_layout(*plan, M, N);
  const bool need_y = grad_y != nullptr, need_x = grad_w != nullptr || grad_x != nullptr;
  ExecArgs ay{}, ax{};
  ay.plan = ax.plan = plan;
  ay.stream = ax.stream = sm;
  ay.lay = &ly;
  ay.ws = wsc;
  ay.x = x;
  ay.y = y;
  ay.w = w;
  ay.deriv = true;
  ay.dout = Dy;
  ay.ldd = ldd;
  ax.lay = &lx;
  ax.ws = wsc + bo.lx;
  ax.x = y;
  ax.y = x;
  ax.w = grad_s;
  ax.ldd = ldd;
  hipError_t e = hipSuccess;
  if (need_y) {
    mark(plan, sm, ST_MISC);
    e = launch_fill_zero(Dy, M * ldd, sm);
    if (e == hipSuccess) e = launch_weight_prep(ay, nullptr);
  }
  if (e == hipSuccess && need_x) {
    mark(plan, sm, ST_MISC);
    if (grad_x) e = launch_fill_zero(Dx, N * ldd, sm);
    if (e == hipSuccess) e = launch_weight_prep(ax, nullptr);
  }
  if (e == hipSuccess && (need_y ? ly : lx).presplit) e = launch_split_points(need_y ? ay : ax);
  for (int32_t p0 = 0; p0 < plan->P && e == hipSuccess; p0 += ly.B) {
    ay.p0 = ax.p0 = p0;
    ay.nsl = ax.nsl = std::min(ly.B, plan->P - p0);
    e = launch_projection(need_y ? ay : ax);
    if (e == hipSuccess) e = launch_slice_setup(need_y ? ay : ax);
    if (e == hipSuccess && need_y && need_x) {
      // Z of (x, y) from Z of (y, x): rows of L floats, the first M columns of each row
      // become the last M, and the per-block bound partials carry over
      mark(plan, sm, ST_MISC);
      const size_t row = (size_t)ly.L * sizeof(float);
      const char *zy = wsc + ly.off_z;
      char *zx = ax.ws + lx.off_z;
      e = hipMemcpy2DAsync(zx, row, zy + (size_t)M * sizeof(float), row, (size_t)N * sizeof(float), ay.nsl,
                           hipMemcpyDeviceToDevice, sm);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(zx + (size_t)N * sizeof(float), row, zy, row, (size_t)M * sizeof(float), ay.nsl,
                             hipMemcpyDeviceToDevice, sm);
      if (e == hipSuccess)
        e = hipMemcpyAsync(ax.ws + lx.off_bounds_part, wsc + ly.off_bounds_part,
                           (size_t)projection_blocks(*plan, ly.L, ay.nsl) * ay.nsl * 2 * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, sm);
      if (e == hipSuccess) e = launch_slice_setup(ax);
    }
    if (e == hipSuccess && need_y) e = post_projection(ay, nullptr);
    if (e == hipSuccess && grad_w) {
      ax.deriv = false;
      ax.dout = nullptr;
      e = post_projection(ax, grad_w);
    }
    if (e == hipSuccess && grad_x) {
      // same sources, weights and targets as the dL/dw sums just made: their spread grid
      // partials and sort buckets are reused, only the mode-dependent stages run again
      ax.deriv = true;
      ax.dout = Dx;
      ax.reuse_front = grad_w != nullptr;
      e = post_projection(ax, nullptr);
      ax.reuse_front = false;
    }
  }
  if (e == hipSuccess && grad_y) {
    mark(plan, sm, ST_BACKPROJ);
    e = launch_backproject(*plan, Dy, ldd, M, grad_s, invP, grad_y, sm);
  }
  if (e == hipSuccess && grad_x) {
    mark(plan, sm, ST_BACKPROJ);
    e = launch_backproject(*plan, Dx, ldd, N, w, invP, grad_x, sm);
  }
  mark(plan, sm, -1);
  note_use(plan, sm);
  if (prev != plan->params.device) (void)hipSetDevice(prev);
  if (e != hipSuccess) return fail(KSUM_EDEVICE, std::string("HIP launch failed: ") + hipGetErrorString(e));
  return KSUM_OK;
}

static const char *kStageNames[ST_COUNT] = {
    "misc", "project", "setup", "ndft_adjoint", "ndft_forward", "nfft_spread", "nfft_grid",
    "nfft_interp", "sort_hist", "sort_scan", "sort_scatter", "sort_group", "accumulate", "sort_fallback",
    "backproject", "split_points"};

int32_t ksum_stage_count(void) { return ST_COUNT; }

const char *ksum_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : "";
}

ksum_status ksum_set_timing(ksum_plan *plan, int32_t enable) {
  if (!plan) return fail(KSUM_EINVAL, "plan is NULL");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(plan->params.device);
  (void)hipDeviceSynchronize();
  free_timer(plan);
  ksum_status st = KSUM_OK;
  if (enable) {
    Timer *t = new (std::nothrow) Timer();
    if (!t) {
      st = fail(KSUM_ENOMEM, "host allocation failed");
    } else {
      t->device = plan->params.device;
      t->ev.resize(kTimerEvents);
      t->ids.resize(kTimerEvents);
      for (auto &e : t->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
          e = nullptr;
          st = fail(KSUM_EDEVICE, "hipEventCreate failed");
          break;
        }
      }
      if (st != KSUM_OK) {
        for (hipEvent_t e : t->ev)
          if (e) (void)hipEventDestroy(e);
        delete t;
      } else {
        plan->timer = t;
      }
    }
  }
  (void)hipSetDevice(prev);
  return st;
}

ksum_status ksum_stage_times(ksum_plan *plan, double *ms_out, int64_t *calls_out) {
  if (!plan || !ms_out) return fail(KSUM_EINVAL, "null argument");
  Timer *t = plan->timer;
  if (!t) return fail(KSUM_EINVAL, "timing is not enabled");
  if (t->used > 0) {
    if (hipEventSynchronize(t->ev[t->used - 1]) != hipSuccess) return fail(KSUM_EDEVICE, "hipEventSynchronize");
    for (int i = 0; i + 1 < t->used; ++i) {
      const int id = t->ids[i];
      if (id < 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t->ev[i], t->ev[i + 1]) != hipSuccess) return fail(KSUM_EDEVICE, "elapsed");
      t->ms[id] += ms;
      t->calls[id] += 1;
    }
    t->used = 0;
  }
  for (int i = 0; i < ST_COUNT; ++i) {
    ms_out[i] = t->ms[i];
    if (calls_out) calls_out[i] = t->calls[i];
  }
  if (t->dropped > 0) {
    const long long n = t->dropped;
    t->dropped = 0;
    return fail(KSUM_EWORKSPACE, std::to_string(n) + " timing marks were dropped (more than " +
                                     std::to_string(kTimerEvents) + " launches between two reads); the times "
                                     "returned miss them");
  }
  return KSUM_OK;
}

}  // extern "C"
