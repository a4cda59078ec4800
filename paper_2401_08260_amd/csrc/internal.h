// Internal declarations of the ksum library: plan, per-slice parameters,
// workspace layout and the kernel launch wrappers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ksum.h"

namespace ksum {

// ---------------------------------------------------------------------------
// Compile-time limits
// ---------------------------------------------------------------------------
constexpr int kMaxTaps = 16;        // 2 * window_m, window_m <= 8
constexpr int kMaxPolyDeg = 13;     // degree of the per-tap window polynomials
constexpr int kGemmBK = 16;         // K step of the projection GEMM (d is padded to it)
constexpr int kGemmBM = 128;        // slices per GEMM tile (P is padded to it)
constexpr int kGemmBlocksPerCU = 3; // persistent projection blocks per CU
constexpr int kMaxBatch = 1024;     // slices per batch (per-block min / max live in LDS)
constexpr int kSortChunkMax = 64;   // chunks per slice in the bucket histogram / scatter, at most
constexpr int kSortChunkLen = 24576; // entries per chunk aimed at: two of the scatter's largest tiles
constexpr int kNfftPPL = 128;       // sources per lane in an NFFT spread block
constexpr int kSortCap = 4096;      // elements a bucket group may hold to be sorted in LDS
constexpr int kSortHalf = kSortCap / 2;

// Kaiser-Bessel window as per-tap polynomials in the fractional grid offset:
// tap j of a point at grid position u = n x (i0 = floor(u), fr = u - i0) sits on
// cell i0 - m + 1 + j and has weight phi((fr + m - 1 - j)/n) ~= sum_q c[j][q] (fr - 1/2)^q.
struct WindowPoly {
  int32_t taps;                     // 2 m
  int32_t deg;                      // polynomial degree
  float c[kMaxTaps][kMaxPolyDeg + 1];
};

// Per-slice parameters computed on the device from the projection bounds.
struct SliceParams {
  double cmin, cmax;      // bounds of the slice's projections (FP32 values as doubles)
  double cmid;            // (cmin + cmax) / 2
  double tau;             // 2T / (cmax - cmin)   (Fourier paths)
  float fcmin;            // cmin as float (bucket map and rescaling)
  float inv_width;        // buckets per unit length (sort path)
  float ftau;             // tau as float
  float shift;            // -T (x~ = tau (x - cmin) - T)
  int32_t eS;             // fixed-point exponent of sum v (z - cmid)
  int32_t pad;
};

// Kernel stages that can be timed with HIP events (ksum_set_timing).
enum StageId {
  ST_MISC = 0, ST_PROJECT, ST_SETUP, ST_NDFT_ADJOINT, ST_NDFT_FORWARD, ST_NFFT_SPREAD, ST_NFFT_GRID,
  ST_NFFT_INTERP, ST_SORT_HIST, ST_SORT_SCAN, ST_SORT_SCATTER, ST_SORT_GROUP, ST_ACCUMULATE,
  ST_SORT_FALLBACK, ST_BACKPROJ, ST_SPLIT_POINTS, ST_COUNT
};

constexpr int kTimerEvents = 16384;   // timing marks held between two reads of the stage times

struct Timer {
  int device = 0;
  std::vector<hipEvent_t> ev;
  std::vector<int> ids;
  int used = 0;
  long long dropped = 0;   // marks that found every event in use since the last read
  double ms[ST_COUNT] = {};
  long long calls[ST_COUNT] = {};
};

}  // namespace ksum

// The opaque plan of the C ABI.
struct ksum_plan {
  int32_t d = 0, P = 0;
  ksum_kernel kernel = KSUM_GAUSSIAN;
  ksum_params params{};          // resolved (no zero "defaults" left), directions pointer cleared
  int32_t method = 0;            // resolved ksum_method of the smooth part (NDFT/NFFT) or SORT
  bool use_sort = false;         // a sort pass (NEGDIST, LAPLACIAN)
  bool use_fourier = false;      // a Fourier pass (GAUSSIAN, LAPLACIAN)
  int32_t d_pad = 0, P_pad = 0;
  int32_t K = 0;                 // largest |k| of the symmetric coefficient set
  int32_t n_grid = 0;            // NFFT grid size
  double cd = 0;                 // c_d
  double sort_const = 0;         // constant of the sorted negative-distance part
  double gauss_logc = 0;         // log(d pi / sqrt(2)) - lgamma((d+2)/2)
  double matern_c3 = 0;          // sqrt(3 pi) Gamma(d/2 + 3/2) / Gamma(d/2) (Matern, nu = 3/2)
  int32_t lap_L = 0;             // samples of the tapered-coefficient recipe (Laplacian, Matern)
  std::vector<double> dirs;      // host directions, P x d
  ksum::WindowPoly poly{};
  // device tables
  float *d_dirs = nullptr;       // [P_pad][d_pad] FP32, zero padded
  uint16_t *d_dirs_hi = nullptr; // [P_pad][d_pad] bf16 hi half of the FP32 directions (split-BF16)
  uint16_t *d_dirs_lo = nullptr; // [P_pad][d_pad] bf16 lo half (split-BF16)
  uint16_t *d_dirs_tiled = nullptr; // [d_pad / 16][P_pad][32] step-tiled hi / lo (split-BF16, P > 256)
  float *d_dirsT = nullptr;      // [d][Pk] FP32 transposed directions (backward), Pk = P rounded up to 16
  int32_t Pk = 0;
  float *d_deconv = nullptr;     // [K+1] 1 / (n phihat(k))^2 (NFFT)
  float2 *d_twiddle = nullptr;   // [n_grid] exp(-2 pi i j / n)
  double *d_costab = nullptr;    // [lap_L] cos(2 pi j / lap_L)
  ksum::Timer *timer = nullptr;  // stage timing (diagnostic), null when off
  // Completion of the plan's work for ksum_plan_destroy: one event per stream that ran
  // the plan, re-recorded after each call on that stream.  Streams beyond the slots set
  // use_overflow, and destroy then waits for the whole device.
  static constexpr int kUseSlots = 32;
  std::mutex use_mu;
  hipStream_t use_stream[kUseSlots] = {};
  hipEvent_t use_event[kUseSlots] = {};
  int n_use = 0;
  bool use_overflow = false;
};

namespace ksum {

void set_error(const std::string &msg);

// ---------------------------------------------------------------------------
// Workspace layout for one execution (all offsets 256-byte aligned)
// ---------------------------------------------------------------------------
struct Layout {
  int64_t N = 0, M = 0, L = 0;   // sources, targets, L = M + N
  int32_t B = 0;                 // slices per batch
  int32_t nb = 0;                // buckets per slice (sort path)
  int32_t sort_groups = 0;       // group slots per slice (sort path)
  int32_t sort_nch = 0;          // chunks per slice of the histogram and the scatter
  int64_t sort_chunk = 0;        // entries per chunk (the last one may hold fewer)
  int32_t ndft_chunks = 0;       // source chunks per slice (NDFT)
  int32_t nfft_chunks = 0;       // source chunks per slice (NFFT spread)
  int32_t win_lo = 0, win_cells = 0;   // NFFT cells touched: [win_lo, win_lo + win_cells)
  size_t off_misc = 0;           // double[8]: sum|w| and scales
  size_t off_wpart = 0;          // double[kWsumBlocks]
  size_t off_params = 0;         // SliceParams[B]
  size_t off_bounds = 0;         // uint32[B][2]
  size_t off_counter = 0;        // uint32[16] tile queue heads of the projection
  size_t off_bounds_part = 0;    // uint32[blocks][B][2] per-block min / max of the projection
  size_t off_z = 0;              // float[B][L]
  size_t off_t1 = 0;             // float[B][M]
  size_t off_t2 = 0;             // float[B][M]
  size_t off_sacc = 0;           // double[M]
  size_t off_coef = 0;           // float[B][K+1]
  size_t off_fpart = 0;          // NDFT float2[B][chunks][K+1] or NFFT float[B][chunks][win_cells]
  size_t off_grid = 0;           // float[B][n_grid]
  size_t off_lapv = 0;           // double[B][lap_L] samples of the Laplacian recipe
  size_t off_wf = 0;             // float[N] weights converted from FP64 input
  size_t off_hcnt = 0;           // uint32[B][sort_nch][nb]
  size_t off_hsum = 0;           // int64[B][sort_nch][nb][2]
  size_t off_bpre = 0;           // int64[B][nb][2]  exclusive bucket prefix of (A, S)
  size_t off_boff = 0;           // uint32[B][nb + 1] bucket offsets
  size_t off_tot = 0;            // int64[B][2]      slice totals (A, S)
  size_t off_keys = 0;           // uint64[B][L] bucketed (key | index << 32)
  size_t off_keys2 = 0;          // uint64[B][L] scratch of the large-group sort
  size_t off_desc = 0;           // int4[B][sort_groups] group descriptors
  size_t off_fail = 0;           // uint32 count (+63 pad) and uint32[B][sort_groups] fallback list
  size_t off_flag = 0;           // uint32 non-finite input flag (opt-in check)
  bool presplit = false;         // the union is split to bf16 hi / lo once per call (split_tiled plans)
  int64_t split_rows = 0;        // L rounded up to whole 256-point tiles
  size_t off_split = 0;          // step-tiled split points [d_pad / 16][split_rows][32] bf16
  size_t total = 0;
};

constexpr int kWsumBlocks = 64;

// Step-tiled split-BF16 operands (directions and pre-split points): per step of 16
// contraction indices s and per row r, 64 bytes holding four 16-byte chunks, c = 0, 1
// the hi values of indices 16 s + 8 c .. + 7 and c = 2, 3 the lo values, chunk c in
// slot c ^ tile_swz(r).  A step of 256 consecutive rows is one contiguous 16 KB block.
__host__ __device__ inline int tile_swz(int64_t r) { return (int)(((r >> 1) ^ (r >> 3)) & 3); }

// Split-BF16 plans with more than 8 tiles of 256 slices keep step-tiled directions and
// split the points once per call into the same layout.  The split pass costs about
// as much as 8 slice tiles save by being fed by it.
constexpr int kTiledMinP = 8 * 2 * kGemmBM + 1;
inline bool split_tiled(const ksum_plan &pl) { return pl.params.precision == KSUM_SPLIT_BF16 && pl.P >= kTiledMinP; }

// batch > 0 sets the slices per batch (at most the plan's own batch size) in place of the plan's;
// allow_presplit = false leaves out the region of the once-per-call split of the points
Layout make_layout(const ksum_plan &plan, int64_t N, int64_t M, int32_t batch = 0, bool allow_presplit = true);

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files).  All take the batch's first
// slice p0 and its size nb_slices; pointers are device pointers.
// ---------------------------------------------------------------------------
struct ExecArgs {
  const ksum_plan *plan;
  const Layout *lay;
  char *ws;
  hipStream_t stream;
  int32_t p0, nsl;        // batch: slices [p0, p0 + nsl)
  const void *x, *y;      // FP32 or FP64 points
  bool f64in;
  const float *w;         // FP32 weights
  bool want_perm;         // order ties by union index
  int32_t *perm_out;      // [P][L] or null
  float *t_out;           // [P][M] or null (probe)
  bool deriv;             // derivative sums instead of sums (backward)
  bool reuse_front;       // the spread grid partials and the sort path's buckets (keys, bucket
                          // prefixes, group descriptors) of this workspace are current for this
                          // batch: only the stages after them run (sums that differ in mode only)
  float *dout;            // derivative mode: [M][ldd] per-target, per-slice derivative sums
  int64_t ldd;
};

template <typename T> inline T *wsp(const ExecArgs &a, size_t off) {
  return reinterpret_cast<T *>(a.ws + off);
}

// Records a timing event on the execution stream: the interval up to the next
// mark is attributed to `stage` (stage < 0 closes the interval).
inline void mark(const ksum_plan *plan, hipStream_t stream, int stage) {
  Timer *t = plan->timer;
  if (!t) return;
  if (t->used >= (int)t->ev.size()) {
    ++t->dropped;
    return;
  }
  if (hipEventRecord(t->ev[t->used], stream) == hipSuccess) t->ids[t->used++] = stage;
}

inline void mark(const ExecArgs &a, int stage) { mark(a.plan, a.stream, stage); }

hipError_t launch_weight_prep(const ExecArgs &a, const double *w64);
hipError_t launch_projection(const ExecArgs &a);
struct GemmCtl;
hipError_t launch_projection_bf16x3(const ExecArgs &a, GemmCtl g);
hipError_t launch_split_points(const ExecArgs &a);
int projection_bf16x3_blocks(int64_t L, int nsl);
int projection_blocks(const ksum_plan &plan, int64_t L, int nsl);
hipError_t launch_slice_setup(const ExecArgs &a);
hipError_t launch_ndft(const ExecArgs &a);
hipError_t launch_nfft(const ExecArgs &a);
hipError_t launch_sort_path(const ExecArgs &a);
hipError_t launch_accumulate(const ExecArgs &a, float *s, bool first, bool last);
hipError_t launch_nfft_interp(const ExecArgs &a, float *s, bool first, bool last);
hipError_t launch_deriv_gather(const ExecArgs &a);
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t stream);
hipError_t launch_check_finite(const void *p, int64_t n, bool f64, uint32_t *flag, hipStream_t stream);
hipError_t launch_backproject(const ksum_plan &plan, const float *D, int64_t ldd, int64_t R, const float *scale,
                              double factor, float *out, hipStream_t stream);

// host tables
void generate_directions(int32_t d, int32_t P, uint64_t seed, double *out);
bool build_window_poly(int m, int n, int oversample, WindowPoly *out, std::string *err);
double kb_phihat(int m, int n, int oversample, int k);

}  // namespace ksum
