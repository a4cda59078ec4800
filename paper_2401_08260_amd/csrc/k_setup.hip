// Per-slice set-up on the device (no host round trip between the projection
// and the 1-D summations):
//   * rescaling of Sec. 3.1: c_min, c_max of the slice, tau = 2T/(c_max - c_min),
//     x~ = tau (x - c_min) - T; a slice whose points all coincide uses
//     c_max - c_min := sigma (any width is valid there);
//   * Gaussian Fourier coefficients c_k = f^_{tau sigma}(k) (Lemma
//     "lem:Fourier_Gauss", evaluated in log space as Sec. 2.2 suggests);
//   * Laplacian smooth-part coefficients (Sec. 3.3): k1(u) = f(|u|/tau) + alpha c_d |u|/tau
//     with its linear term removed, multiplied by the taper
//     W(u) = erfc((|u| - 3/8) * 37) / 2 and integrated over the torus by the
//     trapezoidal rule on L points; the Matern kernel (nu = 3/2) the same recipe on
//     its whole counterpart f(|u|/tau);
//   * the bucket map and fixed-point exponents of the sort path.
// All coefficient arithmetic is FP64.
#include "device_common.h"
#include "internal.h"

namespace ksum {

struct SetupArgs {
  int32_t nsl;
  int32_t kernel;
  int32_t d;
  int32_t K;              // coefficients for k = 0..K
  int32_t nfft;           // 1: fold the NFFT deconvolution into the table
  int32_t nb;             // buckets (sort path)
  int32_t lap_L;
  double T, sigma, eps, gauss_logc, cd, matern_c3;
  uint32_t *bounds;       // [nsl][2] min / max keys (written here from the partials)
  const uint32_t *part;   // [nparts][nsl][2] per-block partials of the projection, or null
  int32_t nparts;
  const double *misc;     // misc[0] = sum |w|
  const float *deconv;    // [K+1]
  const double *costab;   // [lap_L]
  SliceParams *params;
  float *coef;            // [nsl][K+1]
  double *lapv;           // [nsl][lap_L]
  double *bounds_out;     // probe: [P][2] (already offset by p0) or null
};

constexpr int kSeriesTab = 512;   // tabulated term ratios; longer series divide per term
constexpr int kFftHalf = 2048;    // sample counts L up to 2 kFftHalf (powers of two) take the FFT

// Term ratios of the counterpart series, one table per chain (computed once per block):
//  Laplacian (Table "tab:kernels"), a = alpha t: the even and odd chains of
//    f(t) = sum_n (-a)^n sqrt(pi) Gamma((n+d)/2) / (n! Gamma(d/2) Gamma((n+1)/2)) follow
//    T_{n+2} = T_n a^2 (n+d) / ((n+1)^2 (n+2)), T_0 = 1, T_1 = -a c_d;
//  Matern nu = 3/2 (appendix), x = t / beta, z = 3 x^2 / 4:
//    f = 1F2(d/2; 1/2, -1/2; z) + c3 x^3 1F2(d/2 + 3/2; 2, 5/2; z), a 1F2 term ratio being
//    (a + n) z / ((b1 + n) (b2 + n) (n + 1)).
struct SeriesTab {
  double r0[kSeriesTab], r1[kSeriesTab];
};

__device__ __forceinline__ double lap_r0(int n, int d) {          // even chain, step n -> n + 2
  return (double)(n + d) / ((double)(n + 1) * (double)(n + 1) * (double)(n + 2));
}
__device__ __forceinline__ double lap_r1(int n, int d) {          // odd chain, step n + 1 -> n + 3
  return (double)(n + 1 + d) / ((double)(n + 2) * (double)(n + 2) * (double)(n + 3));
}
__device__ __forceinline__ double mat_r0(int n, int d) {
  return (0.5 * d + n) / ((0.5 + n) * (n - 0.5) * (n + 1.0));
}
__device__ __forceinline__ double mat_r1(int n, int d) {
  return (0.5 * d + 1.5 + n) / ((2.0 + n) * (2.5 + n) * (n + 1.0));
}

// Laplacian smooth part k1 at a = alpha t: the series with its linear term removed
// (index i of the tables is the step n = 2 i).
__device__ double laplace_k1_series(double a, int d, double cd, const SeriesTab &tb) {
  const double a2 = a * a;
  double te = 1.0, to = -a * cd;
  double even = 1.0, odd3 = 0.0, big = 1.0;
  for (int n = 0; n < 40000; n += 2) {
    const int i = n >> 1;
    te *= a2 * (i < kSeriesTab ? tb.r0[i] : lap_r0(n, d));
    to *= a2 * (i < kSeriesTab ? tb.r1[i] : lap_r1(n, d));
    even += te;
    odd3 += to;
    big = fmax(big, fmax(fabs(te), fabs(to)));
    if (n > 8 && fabs(te) + fabs(to) <= 1e-18 * big) break;
  }
  return even + odd3;
}

// Matern (nu = 3/2) counterpart at x = t / beta.
__device__ double matern32_series(double x, int d, double c3, const SeriesTab &tb) {
  const double z = 0.75 * x * x;
  double ta = 1.0, tb1 = 1.0, sa = 1.0, sb = 1.0, big = 1.0;
  for (int n = 0; n < 40000; ++n) {
    ta *= z * (n < kSeriesTab ? tb.r0[n] : mat_r0(n, d));
    tb1 *= z * (n < kSeriesTab ? tb.r1[n] : mat_r1(n, d));
    sa += ta;
    sb += tb1;
    big = fmax(big, fmax(fabs(ta), fabs(tb1)));
    if (n > 8 && fabs(ta) + fabs(tb1) <= 1e-18 * big) break;
  }
  return sa + c3 * x * x * x * sb;
}

__global__ __launch_bounds__(256) void slice_setup_kernel(SetupArgs a) {
  const int p = blockIdx.x;
  __shared__ SliceParams sp;
  __shared__ uint32_t red[8];
  if (a.part) {
    // min / max of the slice over the projection blocks' partials
    uint32_t lo = 0xffffffffu, hi = 0u;
    for (int b = threadIdx.x; b < a.nparts; b += blockDim.x) {
      lo = min(lo, a.part[((int64_t)b * a.nsl + p) * 2]);
      hi = max(hi, a.part[((int64_t)b * a.nsl + p) * 2 + 1]);
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = lo;
      red[4 + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = blockDim.x >> 6;
      for (int w = 1; w < nw; ++w) {
        red[0] = min(red[0], red[w]);
        red[4] = max(red[4], red[4 + w]);
      }
      a.bounds[2 * p] = red[0];
      a.bounds[2 * p + 1] = red[4];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float fmin = key_float(a.bounds[2 * p]);
    const float fmax = key_float(a.bounds[2 * p + 1]);
    SliceParams q;
    q.cmin = (double)fmin;
    q.cmax = (double)fmax;
    q.cmid = 0.5 * (q.cmin + q.cmax);
    double range = q.cmax - q.cmin;
    const bool degenerate = !(range > 0.0);
    q.fcmin = fmin;
    q.inv_width = degenerate ? 0.f : (float)((double)a.nb / range);
    if (degenerate) range = a.sigma;
    q.tau = 2.0 * a.T / range;
    q.ftau = (float)q.tau;
    q.shift = (float)(-a.T);
    // fixed-point exponent of sum v (z - cmid): 2^eS * sum|w| * max|z - cmid| < 2^61
    const double wsum = a.misc[0];
    const double half = 0.5 * (q.cmax - q.cmin) * (1.0 + 1e-12) + 1e-300;
    int e = 0;
    if (wsum > 0.0) frexp(wsum * half, &e);
    q.eS = 61 - e;
    q.pad = 0;
    a.params[p] = q;
    sp = q;
    if (a.bounds_out) {
      a.bounds_out[2 * p] = q.cmin;
      a.bounds_out[2 * p + 1] = q.cmax;
    }
  }
  __syncthreads();
  if (a.K < 0) return;
  float *coef = a.coef + (int64_t)p * (a.K + 1);
  if (a.kernel == KSUM_GAUSSIAN) {
    const double st = sp.tau * a.sigma;     // f_sigma(u / tau) = f_{tau sigma}(u)
    for (int k = threadIdx.x; k <= a.K; k += blockDim.x) {
      double c;
      if (k == 0) {
        c = (a.d == 1) ? 2.5066282746310002 * st : 0.0;   // sqrt(2 pi) tau sigma
      } else {
        const double z = 19.739208802178716 * st * st * (double)k * (double)k;   // 2 pi^2 s^2 k^2
        c = exp(a.gauss_logc + log(st) - z + 0.5 * (double)(a.d - 1) * log(z));
      }
      if (fabs(c) <= a.eps) c = 0.0;
      if (a.nfft) c *= (double)a.deconv[k];
      coef[k] = (float)c;
    }
    return;
  }
  // Tapered-coefficient recipe (Laplacian smooth part, Matern): samples v_j of the
  // function times the taper on u_j = -1/2 + j/L, then c_k = (1/L) sum_j v_j cos(2 pi k u_j).
  // The samples depend on |u_j| only, so v_{L-j} = v_j: half of them are evaluated.
  __shared__ SeriesTab tab;
  __shared__ union {
    double part[2048];
    double2 z[2][kFftHalf];
  } sh;
  const bool lap = (a.kernel == KSUM_LAPLACIAN);
  for (int i = threadIdx.x; i < kSeriesTab; i += blockDim.x) {
    tab.r0[i] = lap ? lap_r0(2 * i, a.d) : mat_r0(i, a.d);
    tab.r1[i] = lap ? lap_r1(2 * i, a.d) : mat_r1(i, a.d);
  }
  __syncthreads();
  const int L = a.lap_L;
  const int K1 = a.K + 1;
  const bool use_fft = (L & (L - 1)) == 0 && L >= 64 && L <= 2 * kFftHalf && K1 <= L / 2;
  // samples go to LDS for the FFT (as the complex sequence v_{2m} + i v_{2m+1}), else to
  // the workspace
  double *v = use_fft ? reinterpret_cast<double *>(sh.z[0]) : a.lapv + (int64_t)p * L;
  const double inv_scale = 1.0 / (a.sigma * sp.tau);   // alpha / tau, or 1 / (beta tau)
  for (int j = threadIdx.x; j <= L / 2; j += blockDim.x) {
    const double u = -0.5 + (double)j / (double)L;
    const double au = fabs(u);
    const double taper = 0.5 * erfc((au - 0.375) * 37.0);
    const double f = lap ? laplace_k1_series(inv_scale * au, a.d, a.cd, tab)
                         : matern32_series(inv_scale * au, a.d, a.matern_c3, tab);
    v[j] = f * taper;
    if (j > 0 && j < L - j) v[L - j] = f * taper;
  }
  __syncthreads();
  auto finish = [&](int k, double acc) {
    double c = acc / (double)L;
    if (k & 1) c = -c;
    if (fabs(c) <= a.eps) c = 0.0;
    if (a.nfft) c *= (double)a.deconv[k];
    coef[k] = (float)c;
  };
  if (use_fft) {
    // sum_j v_j cos(2 pi k j / L) = Re V_k, V the length-L DFT of the real v: a length-N
    // complex FFT (N = L / 2, radix-2 Stockham in LDS, twiddles from the exact cosine
    // table) of z_m = v_{2m} + i v_{2m+1}, then V_k = E_k + e^{-2 pi i k / L} O_k with
    // E_k = (Z_k + conj Z_{N-k}) / 2 and O_k = (Z_k - conj Z_{N-k}) / (2 i).
    const int N = L / 2, qL = L / 4;
    double2 *x = sh.z[0], *y = sh.z[1];
    for (int Ls = 1; Ls < N; Ls <<= 1) {
      const int tstep = N / (2 * Ls);
      for (int j = threadIdx.x; j < N / 2; j += blockDim.x) {
        const int k = j & (Ls - 1);
        const int ang = 2 * k * tstep;                   // e^{-2 pi i k tstep / N}, in 1/L turns
        const double wc = a.costab[ang], ws = a.costab[(ang - qL + L) % L];
        const double2 A = x[j], B = x[j + N / 2];
        const double2 b = make_double2(B.x * wc + B.y * ws, B.y * wc - B.x * ws);
        const int o = 2 * j - k;
        y[o] = make_double2(A.x + b.x, A.y + b.y);
        y[o + Ls] = make_double2(A.x - b.x, A.y - b.y);
      }
      __syncthreads();
      double2 *tmp = x;
      x = y;
      y = tmp;
    }
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
      const double2 Zk = x[k], Zn = x[(N - k) % N];
      const double ex = 0.5 * (Zk.x + Zn.x);             // Re E_k
      const double ox = 0.5 * (Zk.y + Zn.y);             // Re O_k
      const double oy = -0.5 * (Zk.x - Zn.x);            // Im O_k
      const double c = a.costab[k], s = a.costab[(k - qL + L) % L];
      finish(k, ex + c * ox + s * oy);                   // Re (E_k + (cos - i sin) O_k)
    }
    return;
  }
  // Other sample counts, a direct DFT: c_k = (1/L) sum_j v_j cos(2 pi k u_j) =
  // (-1)^k (1/L) sum_j v_j cos(2 pi k j / L), the cosine by rotation from the exact table
  // value every 64 steps.  The j range of each k is split over S threads (up to 8,
  // K1 S <= 2048), so that every thread runs short, independent rotation chains; the
  // partial sums are added in order.
  const int qL = L / 4;                    // sin(x) = cos(x - pi/2)
  auto dft_range = [&](int k, int j0, int j1) {
    const int kst = k % L;
    const double cr = a.costab[kst], sr = a.costab[(kst - qL + L) % L];
    double acc = 0.0;
    for (int jb = j0; jb < j1; jb += 64) {
      const int idx = (int)(((int64_t)k * jb) % L);
      double c = a.costab[idx], s = a.costab[(idx - qL + L) % L];
      const int je = min(jb + 64, j1);
      for (int j = jb; j < je; ++j) {
        acc += v[j] * c;
        const double cn = c * cr - s * sr;
        s = s * cr + c * sr;
        c = cn;
      }
    }
    return acc;
  };
  const int S = max(1, min(8, 2048 / K1));
  if (S == 1) {
    for (int k = threadIdx.x; k < K1; k += blockDim.x) finish(k, dft_range(k, 0, L));
    return;
  }
  const int span = (L / S + 63) / 64 * 64;
  for (int it = threadIdx.x; it < K1 * S; it += blockDim.x) {
    const int k = it % K1, sidx = it / K1;
    const int j0 = min(L, sidx * span), j1 = min(L, j0 + span);
    sh.part[it] = dft_range(k, j0, j1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K1; k += blockDim.x) {
    double acc = 0.0;
    for (int sidx = 0; sidx < S; ++sidx) acc += sh.part[sidx * K1 + k];
    finish(k, acc);
  }
}

hipError_t launch_slice_setup(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  SetupArgs s{};
  s.nsl = a.nsl;
  s.kernel = pl.kernel;
  s.d = pl.d;
  s.K = pl.use_fourier ? pl.K : -1;
  s.nfft = (pl.method == KSUM_1D_NFFT) ? 1 : 0;
  s.nb = lay.nb;
  s.lap_L = pl.lap_L;
  s.T = pl.params.T;
  s.sigma = pl.params.sigma;
  s.eps = pl.params.coeff_eps;
  s.gauss_logc = pl.gauss_logc;
  s.cd = pl.cd;
  s.matern_c3 = pl.matern_c3;
  s.bounds = wsp<uint32_t>(a, lay.off_bounds);
  s.part = wsp<uint32_t>(a, lay.off_bounds_part);
  s.nparts = projection_blocks(*a.plan, lay.L, a.nsl);
  s.misc = wsp<double>(a, lay.off_misc);
  s.deconv = pl.d_deconv;
  s.costab = pl.d_costab;
  s.params = wsp<SliceParams>(a, lay.off_params);
  s.coef = wsp<float>(a, lay.off_coef);
  s.lapv = wsp<double>(a, lay.off_lapv);
  s.bounds_out = nullptr;
  mark(a, ST_SETUP);
  slice_setup_kernel<<<a.nsl, 256, 0, a.stream>>>(s);
  return hipGetLastError();
}

hipError_t launch_bounds_probe(const ExecArgs &a, double *bounds_out) {
  // re-run the (cheap) parameter part to export the bounds of this batch
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  SetupArgs s{};
  s.nsl = a.nsl;
  s.kernel = pl.kernel;
  s.d = pl.d;
  s.K = -1;
  s.nb = lay.nb;
  s.T = pl.params.T;
  s.sigma = pl.params.sigma;
  s.bounds = wsp<uint32_t>(a, lay.off_bounds);
  s.misc = wsp<double>(a, lay.off_misc);
  s.params = wsp<SliceParams>(a, lay.off_params);
  s.bounds_out = bounds_out + 2 * (int64_t)a.p0;
  mark(a, ST_MISC);
  slice_setup_kernel<<<a.nsl, 64, 0, a.stream>>>(s);
  return hipGetLastError();
}

}  // namespace ksum
