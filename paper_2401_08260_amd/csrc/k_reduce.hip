// Slice average of Algorithm "Sliced Fast Fourier Summation": s_m = (1/P) sum_p t_{m,p}.
// For the Laplacian t = t1 + t2 (smooth part plus sorted part, Sec. 3.3).  The
// slices of a batch are added in order into an FP64 accumulator, so the result
// does not depend on scheduling.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace ksum {

__global__ __launch_bounds__(256) void accumulate_kernel(const float *__restrict__ t1, const float *__restrict__ t2,
                                                         int nsl, int64_t M, double *__restrict__ sacc,
                                                         float *__restrict__ s, float *__restrict__ t_out, int first,
                                                         int last, double invP) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double acc = first ? 0.0 : sacc[m];
  // 8 slices per round: the loads of a round are independent, the additions stay in order
  constexpr int R = 8;
  int p = 0;
  for (; p + R <= nsl; p += R) {
    float v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = t1[(int64_t)(p + q) * M + m];
    if (t2) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] += t2[(int64_t)(p + q) * M + m];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      acc += (double)v[q];
      if (t_out) t_out[(int64_t)(p + q) * M + m] = v[q];
    }
  }
  for (; p < nsl; ++p) {
    float v = t1[(int64_t)p * M + m];
    if (t2) v += t2[(int64_t)p * M + m];
    acc += (double)v;
    if (t_out) t_out[(int64_t)p * M + m] = v;
  }
  if (last) s[m] = (float)(acc * invP);
  else sacc[m] = acc;
}

hipError_t launch_accumulate(const ExecArgs &a, float *s, bool first, bool last) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  const float *t1 = wsp<float>(a, lay.off_t1);
  const float *t2 = (pl.kernel == KSUM_LAPLACIAN) ? wsp<float>(a, lay.off_t2) : nullptr;
  double *sacc = wsp<double>(a, lay.off_sacc);
  float *tout = a.t_out ? a.t_out + (int64_t)a.p0 * lay.M : nullptr;
  const unsigned grid = (unsigned)((lay.M + 255) / 256);
  mark(a, ST_ACCUMULATE);
  accumulate_kernel<<<grid, 256, 0, a.stream>>>(t1, t2, a.nsl, lay.M, sacc, s, tout, first ? 1 : 0,
                                                last ? 1 : 0, 1.0 / (double)pl.P);
  return hipGetLastError();
}

// Derivative mode: the per-slice derivative sums of a batch, slice-major in t1 (plus
// the sorted part t2 of the Laplacian), go to the per-target rows of dout that the
// back-projection reads: dout[m][p0 + p].  64 targets x 16 slices per block through
// LDS, so both the reads and the writes are runs of consecutive addresses.
__global__ __launch_bounds__(256) void deriv_gather_kernel(const float *__restrict__ t1, const float *__restrict__ t2,
                                                           int nsl, int64_t M, float *__restrict__ dout,
                                                           int64_t ldd, int p0) {
  __shared__ float tile[16][65];
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int q0 = blockIdx.y * 16;
  const int t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = r * 4 + (t >> 6), mi = t & 63;
    const int64_t m = m0 + mi;
    float v = 0.f;
    if (q0 + q < nsl && m < M) {
      v = t1[(int64_t)(q0 + q) * M + m];
      if (t2) v += t2[(int64_t)(q0 + q) * M + m];
    }
    tile[q][mi] = v;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = r * 256 + t;
    const int mi = e >> 4, q = e & 15;
    const int64_t m = m0 + mi;
    if (q0 + q < nsl && m < M) dout[m * ldd + p0 + q0 + q] = tile[q][mi];
  }
}

hipError_t launch_deriv_gather(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  // used where t passes through HBM: NDFT (t1, plus the sorted part t2 of the
  // Laplacian) and the negative distance (t1)
  const float *t1 = wsp<float>(a, lay.off_t1);
  const float *t2 = (pl.kernel == KSUM_LAPLACIAN) ? wsp<float>(a, lay.off_t2) : nullptr;
  mark(a, ST_ACCUMULATE);
  dim3 grid((unsigned)((lay.M + 63) / 64), (unsigned)((a.nsl + 15) / 16));
  deriv_gather_kernel<<<grid, 256, 0, a.stream>>>(t1, t2, a.nsl, lay.M, a.dout, a.ldd, a.p0);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(float *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  fill_zero_kernel<<<grid, 256, 0, stream>>>(p, n);
  return hipGetLastError();
}

// Opt-in input check: sets *flag to 1 if any of the n values is NaN or infinite.  The
// flag is cleared by the caller (a fill kernel) before the first check of a call.
template <typename T>
__global__ __launch_bounds__(256) void check_finite_kernel(const T *__restrict__ p, int64_t n,
                                                          uint32_t *__restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) *flag = 1u;
}

hipError_t launch_check_finite(const void *p, int64_t n, bool f64, uint32_t *flag, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  if (f64) check_finite_kernel<double><<<grid, 256, 0, stream>>>(static_cast<const double *>(p), n, flag);
  else check_finite_kernel<float><<<grid, 256, 0, stream>>>(static_cast<const float *>(p), n, flag);
  return hipGetLastError();
}

}  // namespace ksum
