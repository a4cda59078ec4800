// Slice average of Algorithm "Sliced Fast Fourier Summation": s_m = (1/P) sum_p t_{m,p}.
// For the Laplacian t = t1 + t2 (smooth part plus sorted part, Sec. 3.3).  The
// slices of a batch are added in order into an FP64 accumulator, so the result
// does not depend on scheduling.
#include "device_common.h"
#include "internal.h"

namespace ksum {

__global__ __launch_bounds__(256) void accumulate_kernel(const float *__restrict__ t1, const float *__restrict__ t2,
                                                         int nsl, int64_t M, double *sacc, float *s,
                                                         float *t_out, int first, int last, double invP) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double acc = first ? 0.0 : sacc[m];
  for (int p = 0; p < nsl; ++p) {
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

}  // namespace ksum
