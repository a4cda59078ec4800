// Fast Fourier summation of Sec. 3.1 on every slice, after the rescaling
// x~ = tau (x - c_min) - T (Sec. 3.1, "Rescaling"):
//
//   w^_k = sum_n w_n exp(-2 pi i k x~_n)           (adjoint transform)
//   t_m  = sum_k c_k w^_k exp(+2 pi i k y~_m)      (transform at the targets)
//
// with real even coefficients c_k (so t_m = c_0 w^_0 + 2 Re sum_{k>=1} ...).
//
// NDFT: the transforms evaluated directly, O((N+M)|C|) (Sec. 3.1).
// NFFT (the Remark "Non-equispaced FFT" of Sec. 3.1): sources are spread onto an
// oversampled grid of n = sigma_os * n_coeff cells with a Kaiser-Bessel window
// of half-width m, the grid is transformed by an FFT, multiplied by
// c_k / (n phi^(k))^2 (deconvolution of both window passes), transformed back,
// and interpolated at the targets with the same window.  Points only occupy
// [-T, T], so spreading and interpolation touch a window of W cells around 0;
// the spread accumulates into copies of that window in LDS, one per lane or per
// few lanes ([cell][copy] layout: conflict-free, deterministic), then copies and
// chunks are reduced in a fixed order.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace ksum {

// ---------------------------------------------------------------------------
// NDFT
// ---------------------------------------------------------------------------
constexpr int kNdftChunk = 4096;   // sources per adjoint block
constexpr int kNdftKB = 8;         // coefficients per adjoint block (one k-group)

struct FourierArgs {
  int32_t nsl, K, chunks;
  int64_t N, M, L;
  const float *Z;
  const float *w;
  const SliceParams *params;
  const float *coef;       // [nsl][K+1]
  float2 *part;            // NDFT: [nsl][chunks][K+1]
  float *gpart;            // NFFT: [nsl][chunks][W]
  float *gwin;             // NFFT: [nsl][W] interpolation grid window
  float *t;                // [nsl][M]
  // NFFT
  int32_t n, W, lo;        // grid size, window cells, first window cell (may be < 0)
  int32_t share;           // lanes per window copy in the spread (1..64)
  int32_t i0min, i0max;    // clamp of the base cell
  const float2 *twiddle;   // [n]
  WindowPoly poly;
  int32_t deriv;           // derivative sums (coefficients times 2 pi i k, result times tau)
};

// One block per (slice, chunk of sources, group of kNdftKB coefficients): the
// coefficient groups run in parallel, so a small problem still fills the chip.
__global__ __launch_bounds__(256) void ndft_adjoint_kernel(FourierArgs a) {
  __shared__ float2 red[4][kNdftKB];
  const int ng = (a.K + kNdftKB) / kNdftKB;   // k-groups covering 0..K
  const int64_t work = xcd_remap(blockIdx.x, (int64_t)a.nsl * a.chunks * ng);
  if (work < 0) return;
  const int g = (int)(work % ng);
  const int64_t pc = work / ng;
  const int p = (int)(pc / a.chunks), c = (int)(pc % a.chunks);
  const SliceParams sp = a.params[p];
  const float *Zx = a.Z + (int64_t)p * a.L + a.M;
  const int64_t n0 = (int64_t)c * kNdftChunk, n1 = min(a.N, n0 + kNdftChunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  {
    const int kb = g * kNdftKB;
    float re[kNdftKB], im[kNdftKB];
#pragma unroll
    for (int q = 0; q < kNdftKB; ++q) re[q] = im[q] = 0.f;
    for (int64_t i = n0 + threadIdx.x; i < n1; i += 256) {
      const float xt = (Zx[i] - sp.fcmin) * sp.ftau + sp.shift;
      const float wv = a.w[i];
#pragma unroll
      for (int q = 0; q < kNdftKB; ++q) {
        const int k = kb + q;
        float s, co;
        sincospif(2.0f * (float)k * xt, &s, &co);   // exp(-2 pi i k x) = cos - i sin
        re[q] += wv * co;
        im[q] -= wv * s;
      }
    }
#pragma unroll
    for (int q = 0; q < kNdftKB; ++q) {
      const float r = wave_sum(re[q]), m = wave_sum(im[q]);
      if (lane == 0) red[wid][q] = make_float2(r, m);
    }
    __syncthreads();
    if (threadIdx.x < kNdftKB && kb + (int)threadIdx.x <= a.K) {
      const int q = threadIdx.x;
      float2 s = red[0][q];
      for (int w2 = 1; w2 < 4; ++w2) {
        s.x += red[w2][q].x;
        s.y += red[w2][q].y;
      }
      a.part[((int64_t)p * a.chunks + c) * (a.K + 1) + kb + q] = s;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void ndft_forward_kernel(FourierArgs a, int ychunk) {
  extern __shared__ float2 h[];   // [K+1]
  const int nyc = (int)((a.M + ychunk - 1) / ychunk);
  const int64_t work = xcd_remap(blockIdx.x, (int64_t)a.nsl * nyc);
  if (work < 0) return;
  const int p = (int)(work / nyc), c = (int)(work % nyc);
  const SliceParams sp = a.params[p];
  for (int k = threadIdx.x; k <= a.K; k += blockDim.x) {
    float2 s = make_float2(0.f, 0.f);
    const float2 *pp = a.part + (int64_t)p * a.chunks * (a.K + 1) + k;
    for (int q = 0; q < a.chunks; ++q) {
      const float2 v = pp[(int64_t)q * (a.K + 1)];
      s.x += v.x;
      s.y += v.y;
    }
    const float ck = a.coef[(int64_t)p * (a.K + 1) + k];
    const float f = (k == 0) ? ck : 2.0f * ck;   // c_{-k} w^_{-k} is the conjugate term
    h[k] = make_float2(f * s.x, f * s.y);
  }
  __syncthreads();
  const float *Zy = a.Z + (int64_t)p * a.L;
  float *tp = a.t + (int64_t)p * a.M;
  const int64_t m0 = (int64_t)c * ychunk, m1 = min(a.M, m0 + ychunk);
  for (int64_t m = m0 + threadIdx.x; m < m1; m += blockDim.x) {
    const float yt = (Zy[m] - sp.fcmin) * sp.ftau + sp.shift;
    float acc = 0.f;
    if (a.deriv) {
      // d/dy~ Re((hr + i hi) exp(2 pi i k y~)) = -2 pi k (hr sin + hi cos); times tau = dy~/dz
      for (int k = 1; k <= a.K; ++k) {
        float s, co;
        sincospif(2.0f * (float)k * yt, &s, &co);
        acc += (float)k * (h[k].x * s + h[k].y * co);
      }
      tp[m] = -6.283185307179586f * sp.ftau * acc;
    } else {
      for (int k = 0; k <= a.K; ++k) {
        float s, co;
        sincospif(2.0f * (float)k * yt, &s, &co);
        // Re((hr + i hi)(cos + i sin)) = hr cos - hi sin
        acc += h[k].x * co - h[k].y * s;
      }
      tp[m] = acc;
    }
  }
}

hipError_t launch_ndft(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  FourierArgs f{};
  f.nsl = a.nsl;
  f.K = pl.K;
  f.chunks = lay.ndft_chunks;
  f.N = lay.N;
  f.M = lay.M;
  f.L = lay.L;
  f.Z = wsp<float>(a, lay.off_z);
  f.w = a.w;
  f.params = wsp<SliceParams>(a, lay.off_params);
  f.coef = wsp<float>(a, lay.off_coef);
  f.part = wsp<float2>(a, lay.off_fpart);
  f.t = wsp<float>(a, lay.off_t1);
  f.deriv = a.deriv ? 1 : 0;
  mark(a, ST_NDFT_ADJOINT);
  const int ng = (pl.K + kNdftKB) / kNdftKB;
  ndft_adjoint_kernel<<<(unsigned)xcd_grid((int64_t)a.nsl * f.chunks * ng), 256, 0, a.stream>>>(f);
  const int ychunk = 256;   // one target per thread: small problems still fill the chip
  const int nyc = (int)((lay.M + ychunk - 1) / ychunk);
  mark(a, ST_NDFT_FORWARD);
  ndft_forward_kernel<<<(unsigned)xcd_grid((int64_t)a.nsl * nyc), 256, (pl.K + 1) * sizeof(float2),
                        a.stream>>>(f, ychunk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// NFFT
// ---------------------------------------------------------------------------

// Window weights of the 2 MW taps of a point with fractional offset x = fr - 1/2:
// tap j and tap 2 MW - 1 - j are mirror images, poly_{2MW-1-j}(x) = poly_j(-x), so the
// even and odd parts of the first MW polynomials give all taps.
template <int MW, int DEG>
__device__ __forceinline__ void window_taps(const WindowPoly &wp, float x, float (&tap)[2 * MW]) {
  const float x2 = x * x;
#pragma unroll
  for (int j = 0; j < MW; ++j) {
    float e = wp.c[j][DEG - (DEG & 1)];
#pragma unroll
    for (int q = DEG - (DEG & 1) - 2; q >= 0; q -= 2) e = fmaf(e, x2, wp.c[j][q]);
    float o = wp.c[j][DEG - 1 + (DEG & 1)];
#pragma unroll
    for (int q = DEG - 1 + (DEG & 1) - 2; q >= 1; q -= 2) o = fmaf(o, x2, wp.c[j][q]);
    const float xo = x * o;
    tap[j] = e + xo;
    tap[2 * MW - 1 - j] = e - xo;
  }
}

// Spreading of one chunk of 256 x kNfftPPL sources of a slice.  The W-cell window
// is kept in LDS as 256/SH copies ([cell][copy]); SH lanes of a wave share a copy and
// update it one after the other (SH phases in lane order), so every copy sees its
// updates in a fixed order and the result is deterministic.  SH grows with the
// window so that wide windows (the Laplacian's and Matern's T = 1/8) still leave
// room for two blocks per CU.
template <int MW, int DEG, int SH>
__global__ __launch_bounds__(256) void nfft_spread_kernel(FourierArgs a) {
  extern __shared__ float acc[];   // [W][NC]
  constexpr int CW = 64 / SH;      // copies per wave
  constexpr int NC = 256 / SH;     // copies per block
  const int64_t work = xcd_remap(blockIdx.x, (int64_t)a.nsl * a.chunks);
  if (work < 0) return;
  const int p = (int)(work / a.chunks), c = (int)(work % a.chunks);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int copy = wid * CW + lane % CW, phase = lane / CW;
  for (int i = t; i < a.W * NC; i += 256) acc[i] = 0.f;
  __syncthreads();
  const SliceParams sp = a.params[p];
  const float *Zx = a.Z + (int64_t)p * a.L + a.M;
  const int64_t chunk = (int64_t)256 * kNfftPPL;
  const int64_t n0 = (int64_t)c * chunk, n1 = min(a.N, n0 + chunk);
  const float fn = (float)a.n;
  // sources in batches of kSU per thread; the next batch's projections and weights
  // are loaded while the current one is spread
  constexpr int kSU = 4;
  float zn[kSU], wn[kSU];
  auto load = [&](int64_t i, float (&z)[kSU], float (&w)[kSU]) {
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const int64_t iu = i + 256 * u;
      z[u] = iu < n1 ? Zx[iu] : 0.f;
      w[u] = iu < n1 ? a.w[iu] : 0.f;
    }
  };
  load(n0 + t, zn, wn);
  for (int64_t ib = n0 + t; ib < n1; ib += 256 * kSU) {
    float zc[kSU], wc[kSU];
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      zc[u] = zn[u];
      wc[u] = wn[u];
    }
    if (ib + 256 * kSU < n1) load(ib + 256 * kSU, zn, wn);
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      if (ib + 256 * u >= n1) break;
      const float xt = (zc[u] - sp.fcmin) * sp.ftau + sp.shift;
      const float uu = xt * fn;
      int i0 = (int)floorf(uu);
      const float fr = uu - (float)i0;
      i0 = min(max(i0, a.i0min), a.i0max);
      float tap[2 * MW];
      window_taps<MW, DEG>(a.poly, fr - 0.5f, tap);
      const float wv = wc[u];
      // the 2 MW cells of this lane's copy are distinct: read them all, then write
      float *base = acc + (i0 - MW + 1 - a.lo) * NC + copy;
#pragma unroll 1
      for (int ph = 0; ph < SH; ++ph) {
        if (phase == ph) {
          float v[2 * MW];
#pragma unroll
          for (int j = 0; j < 2 * MW; ++j) v[j] = base[j * NC];
#pragma unroll
          for (int j = 0; j < 2 * MW; ++j) base[j * NC] = fmaf(wv, tap[j], v[j]);
        }
      }
    }
  }
  __syncthreads();
  // reduce the copies of every cell in a fixed order: one wave per cell
  float *out = a.gpart + ((int64_t)p * a.chunks + c) * a.W;
  for (int cell = wid; cell < a.W; cell += 4) {
    float s = 0.f;
    for (int l = lane; l < NC; l += 64) s += acc[cell * NC + l];
    s = wave_sum(s);
    if (lane == 0) out[cell] = s;
  }
}

// One slice per block: reduce chunk partials, FFT, diagonal, inverse FFT.
__global__ __launch_bounds__(256) void nfft_grid_kernel(FourierArgs a) {
  extern __shared__ float2 fbuf[];   // [2][n]
  const int p = blockIdx.x;
  const int n = a.n, t = threadIdx.x, lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
  float2 *x = fbuf, *y = fbuf + n;
  for (int i = t; i < n; i += blockDim.x) x[i] = make_float2(0.f, 0.f);
  __syncthreads();
  const float *gp = a.gpart + (int64_t)p * a.chunks * a.W;
  for (int cell = wid; cell < a.W; cell += nw) {
    float s = 0.f;
    for (int q = lane; q < a.chunks; q += 64) s += gp[(int64_t)q * a.W + cell];
    s = wave_sum(s);
    if (lane == 0) {
      int gi = (a.lo + cell) % n;
      if (gi < 0) gi += n;
      x[gi].x = s;
    }
  }
  __syncthreads();
  // forward FFT (radix-2 Stockham): g^_k = sum_l g_l exp(-2 pi i k l / n)
  for (int Ls = 1; Ls < n; Ls <<= 1) {
    const int tstep = n / (2 * Ls);
    for (int j = t; j < n / 2; j += blockDim.x) {
      const int k = j & (Ls - 1);
      const float2 A = x[j], Bv = x[j + n / 2];
      const float2 wv = a.twiddle[k * tstep];
      const float2 b = make_float2(Bv.x * wv.x - Bv.y * wv.y, Bv.x * wv.y + Bv.y * wv.x);
      const int o = 2 * j - k;
      y[o] = make_float2(A.x + b.x, A.y + b.y);
      y[o + Ls] = make_float2(A.x - b.x, A.y - b.y);
    }
    __syncthreads();
    float2 *tmp = x; x = y; y = tmp;
  }
  // diagonal: c_k / (n phi^(k))^2 for |k| <= K, zero elsewhere
  const float *cf = a.coef + (int64_t)p * (a.K + 1);
  for (int j = t; j < n; j += blockDim.x) {
    const int k = (j < n / 2) ? j : j - n;
    const int ak = k < 0 ? -k : k;
    const float f = (ak <= a.K) ? cf[ak] : 0.f;
    if (a.deriv) {
      // times 2 pi i k: the inverse transform is then the derivative in y~
      const float c = 6.283185307179586f * (float)k * f;
      x[j] = make_float2(-x[j].y * c, x[j].x * c);
    } else {
      x[j] = make_float2(x[j].x * f, x[j].y * f);
    }
  }
  __syncthreads();
  // inverse FFT: G_l = sum_k h_k exp(+2 pi i k l / n)
  for (int Ls = 1; Ls < n; Ls <<= 1) {
    const int tstep = n / (2 * Ls);
    for (int j = t; j < n / 2; j += blockDim.x) {
      const int k = j & (Ls - 1);
      const float2 A = x[j], Bv = x[j + n / 2];
      const float2 wv = a.twiddle[k * tstep];   // conjugated below
      const float2 b = make_float2(Bv.x * wv.x + Bv.y * wv.y, Bv.y * wv.x - Bv.x * wv.y);
      const int o = 2 * j - k;
      y[o] = make_float2(A.x + b.x, A.y + b.y);
      y[o + Ls] = make_float2(A.x - b.x, A.y - b.y);
    }
    __syncthreads();
    float2 *tmp = x; x = y; y = tmp;
  }
  float *gw = a.gwin + (int64_t)p * a.W;
  for (int cell = t; cell < a.W; cell += blockDim.x) {
    int gi = (a.lo + cell) % n;
    if (gi < 0) gi += n;
    gw[cell] = x[gi].x;
  }
}

// Interpolation at the targets fused with the slice average (Algorithm
// "Sliced Fast Fourier Summation", last step): every block owns 256 targets,
// stages the grid windows of a sub-batch of slices in LDS and adds
// t_{m,p} (plus the sorted part t2 of the Laplacian) over the slices in order in
// FP64, so t never goes through HBM.  Optionally writes the per-slice t (probe).
struct AccumArgs {
  const float *t2;        // [nsl][M] sorted part (Laplacian) or null
  double *sacc;           // [M] accumulator across batches
  float *s;               // [M] output
  float *t_out;           // [nsl][M] per-slice sums (probe) or null
  int first, last;
  double invP;
  float *dout;            // derivative mode: dout[m * ldd + p0 + p] = tau t'(y~) + t2, no average
  int64_t ldd;
  int p0;
};

// One target per thread.  A block stages the grid windows and the rescaling of a
// sub-batch of sb slices in LDS (8 loads in flight per thread), and each thread
// loads the projections (and t2) of the next kIU slices while it evaluates the
// current ones, so that many loads are in flight.
constexpr int kIU = 8;

template <int MW, int DEG, bool DERIV>
__global__ __launch_bounds__(256) void nfft_interp_accum_kernel(FourierArgs a, AccumArgs c, int sb) {
  extern __shared__ float G[];   // [sb][W] window values, then [sb][3] (fcmin, ftau, shift)
  const int64_t nblk = (a.M + 255) / 256;
  const int64_t work = xcd_remap(blockIdx.x, nblk);
  if (work < 0) return;
  const int64_t m = work * 256 + threadIdx.x;
  const bool live = m < a.M;
  const float fn = (float)a.n;
  float *SP = G + (size_t)sb * a.W;
  // the running FP64 sum continues from the previous batch, so the additions run in
  // slice order whatever the batch size
  double acc = (!DERIV && live && !c.first) ? c.sacc[m] : 0.0;
  for (int pb = 0; pb < a.nsl; pb += sb) {
    const int np = min(sb, a.nsl - pb);
    __syncthreads();
    const int nw = np * a.W;
    const float *gsrc = a.gwin + (int64_t)pb * a.W;
    for (int i0 = threadIdx.x; i0 < nw; i0 += 256 * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (i0 + 256 * u < nw) ? gsrc[i0 + 256 * u] : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + 256 * u < nw) G[i0 + 256 * u] = v[u];
    }
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
      const SliceParams sp = a.params[pb + q];
      SP[3 * q] = sp.fcmin;
      SP[3 * q + 1] = sp.ftau;
      SP[3 * q + 2] = sp.shift;
    }
    __syncthreads();
    // batches of kIU slices; the loads of the next batch are issued before the
    // current one is evaluated
    float zn[kIU], t2n[kIU];
    auto load = [&](int q0, float (&z)[kIU], float (&t2)[kIU]) {
#pragma unroll
      for (int u = 0; u < kIU; ++u) {
        const int p = pb + q0 + u;
        const bool ok = live && q0 + u < np;
        z[u] = ok ? a.Z[(int64_t)p * a.L + m] : 0.f;
        t2[u] = (ok && c.t2) ? c.t2[(int64_t)p * a.M + m] : 0.f;
      }
    };
    load(0, zn, t2n);
    for (int q0 = 0; q0 < np; q0 += kIU) {
      float zv[kIU], t2v[kIU];
#pragma unroll
      for (int u = 0; u < kIU; ++u) {
        zv[u] = zn[u];
        t2v[u] = t2n[u];
      }
      if (q0 + kIU < np) load(q0 + kIU, zn, t2n);
#pragma unroll
      for (int u = 0; u < kIU; ++u) {
        const int q = q0 + u;
        if (q >= np || !live) break;
        const int p = pb + q;
        const float ftau = SP[3 * q + 1];
        const float yt = (zv[u] - SP[3 * q]) * ftau + SP[3 * q + 2];
        const float uu = yt * fn;
        int i0 = (int)floorf(uu);
        const float fr = uu - (float)i0;
        i0 = min(max(i0, a.i0min), a.i0max);
        float tap[2 * MW];
        window_taps<MW, DEG>(a.poly, fr - 0.5f, tap);
        const float *gb = G + q * a.W + (i0 - MW + 1 - a.lo);
        float tv = 0.f;
#pragma unroll
        for (int j = 0; j < 2 * MW; ++j) tv = fmaf(gb[j], tap[j], tv);
        if (DERIV) tv *= ftau;
        tv += t2v[u];
        if (c.t_out) c.t_out[(int64_t)p * a.M + m] = tv;
        if (DERIV) c.dout[m * c.ldd + c.p0 + p] = tv;
        acc += (double)tv;
      }
    }
  }
  if (DERIV || !live) return;
  if (c.last) c.s[m] = (float)(acc * c.invP);
  else c.sacc[m] = acc;
}

template <int MW, int DEG, int SH>
static void launch_spread_sh(const FourierArgs &f, const ExecArgs &a, unsigned gs) {
  const size_t lds = (size_t)f.W * (256 / SH) * sizeof(float);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void *)nfft_spread_kernel<MW, DEG, SH>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  nfft_spread_kernel<MW, DEG, SH><<<gs, 256, lds, a.stream>>>(f);
}

template <int MW, int DEG>
static void launch_nfft_m(const FourierArgs &f, const ExecArgs &a) {
  const unsigned gs = (unsigned)xcd_grid((int64_t)a.nsl * f.chunks);
  const size_t grid_lds = 2 * (size_t)f.n * sizeof(float2);
  if (grid_lds > 65536)
    (void)hipFuncSetAttribute((const void *)nfft_grid_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)grid_lds);
  if (!a.reuse_front) {   // the spread does not depend on the derivative mode
    mark(a, ST_NFFT_SPREAD);
    switch (f.share) {
      case 1: launch_spread_sh<MW, DEG, 1>(f, a, gs); break;
      case 2: launch_spread_sh<MW, DEG, 2>(f, a, gs); break;
      case 4: launch_spread_sh<MW, DEG, 4>(f, a, gs); break;
      case 8: launch_spread_sh<MW, DEG, 8>(f, a, gs); break;
      case 16: launch_spread_sh<MW, DEG, 16>(f, a, gs); break;
      case 32: launch_spread_sh<MW, DEG, 32>(f, a, gs); break;
      default: launch_spread_sh<MW, DEG, 64>(f, a, gs); break;
    }
  }
  mark(a, ST_NFFT_GRID);
  nfft_grid_kernel<<<a.nsl, 256, grid_lds, a.stream>>>(f);
}

// Lanes per window copy of the spread: the smallest power of two that keeps a
// 256-thread block's copies within 80 KB (two blocks per CU: fewer ordered phases
// pay more than a third and fourth block would); 0 if even 64 lanes per copy (4
// copies) do not fit 64 KB.
int nfft_share_for(int W) {
  for (int sh = 1; sh <= 64; sh <<= 1)
    if ((size_t)W * (256 / sh) * sizeof(float) <= 80 * 1024) return sh;
  return ((size_t)W * 4 * sizeof(float) <= 64 * 1024) ? 64 : 0;
}

static FourierArgs nfft_args(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  FourierArgs f{};
  f.nsl = a.nsl;
  f.K = pl.K;
  f.chunks = lay.nfft_chunks;
  f.N = lay.N;
  f.M = lay.M;
  f.L = lay.L;
  f.Z = wsp<float>(a, lay.off_z);
  f.w = a.w;
  f.params = wsp<SliceParams>(a, lay.off_params);
  f.coef = wsp<float>(a, lay.off_coef);
  f.gpart = wsp<float>(a, lay.off_fpart);
  f.gwin = wsp<float>(a, lay.off_grid);
  f.t = wsp<float>(a, lay.off_t1);
  f.n = pl.n_grid;
  f.W = lay.win_cells;
  f.lo = lay.win_lo;
  f.share = nfft_share_for(lay.win_cells);
  const int m = pl.params.window_m;
  f.i0min = lay.win_lo + m - 1;
  f.i0max = lay.win_lo + lay.win_cells - 1 - m;
  f.twiddle = pl.d_twiddle;
  f.poly = pl.poly;
  f.deriv = a.deriv ? 1 : 0;
  return f;
}

hipError_t launch_nfft(const ExecArgs &a) {
  const FourierArgs f = nfft_args(a);
  switch (a.plan->params.window_m) {
    case 2: launch_nfft_m<2, 9>(f, a); break;
    case 3: launch_nfft_m<3, 9>(f, a); break;
    case 4: launch_nfft_m<4, 7>(f, a); break;
    case 5: launch_nfft_m<5, 7>(f, a); break;
    case 6: launch_nfft_m<6, 7>(f, a); break;
    case 7: launch_nfft_m<7, 7>(f, a); break;
    case 8: launch_nfft_m<8, 7>(f, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MW, int DEG>
static void launch_interp_m(const FourierArgs &f, const AccumArgs &c, const ExecArgs &a) {
  const unsigned grid = (unsigned)xcd_grid((f.M + 255) / 256);
  const int sb = std::max(1, std::min(f.nsl, (int)(32768 / ((f.W + 3) * (int)sizeof(float)))));
  const size_t lds = (size_t)sb * (f.W + 3) * sizeof(float);
  mark(a, ST_NFFT_INTERP);
  if (c.dout)
    nfft_interp_accum_kernel<MW, DEG, true><<<grid, 256, lds, a.stream>>>(f, c, sb);
  else
    nfft_interp_accum_kernel<MW, DEG, false><<<grid, 256, lds, a.stream>>>(f, c, sb);
}

hipError_t launch_nfft_interp(const ExecArgs &a, float *s, bool first, bool last) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  const FourierArgs f = nfft_args(a);
  AccumArgs c{};
  c.t2 = (pl.kernel == KSUM_LAPLACIAN) ? wsp<float>(a, lay.off_t2) : nullptr;
  c.sacc = wsp<double>(a, lay.off_sacc);
  c.s = s;
  c.t_out = a.t_out ? a.t_out + (int64_t)a.p0 * lay.M : nullptr;
  c.first = first ? 1 : 0;
  c.last = last ? 1 : 0;
  c.invP = 1.0 / (double)pl.P;
  c.dout = a.deriv ? a.dout : nullptr;
  c.ldd = a.ldd;
  c.p0 = a.p0;
  switch (pl.params.window_m) {
    case 2: launch_interp_m<2, 9>(f, c, a); break;
    case 3: launch_interp_m<3, 9>(f, c, a); break;
    case 4: launch_interp_m<4, 7>(f, c, a); break;
    case 5: launch_interp_m<5, 7>(f, c, a); break;
    case 6: launch_interp_m<6, 7>(f, c, a); break;
    case 7: launch_interp_m<7, 7>(f, c, a); break;
    case 8: launch_interp_m<8, 7>(f, c, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Degree of the per-tap window polynomials: the smallest that fits the Kaiser-Bessel
// taps to within 5e-8 of phi(0) for oversampling 2..8 (narrow windows are steeper per
// cell).  With FP32 coefficients no degree gets below about 2e-8.
int window_degree_for(int m) { return m <= 3 ? 9 : 7; }

}  // namespace ksum
