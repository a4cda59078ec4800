// Projection GEMM of the sliced summation: Z[p][l] = <xi_p, u_l> for the union
// u = (y_1..y_M, x_1..x_N) (targets first, as in the union of Sec. 3.2), with
// per-slice minimum and maximum of the projections (the c_min, c_max of the
// rescaling in Sec. 3.1, and the bucket range of the sort path).
//
// FP32 matrix cores: v_mfma_f32_32x32x2f32.  A tile of 128 slices x 128 points
// per workgroup (4 waves, 2 x 2, each 64 x 64 = 2 x 2 MFMA blocks), K step 16
// double buffered in LDS.  Lane l of an MFMA holds A[l % 32][k] and B[k][l % 32]
// with k = 8 (l / 32) + s for step s = 0..7 of a K-block of 16 (any assignment of
// the contraction index works as long as A and B agree), so a lane reads 8
// consecutive floats of its row with two 16-byte LDS loads.
#include "device_common.h"
#include "internal.h"

namespace ksum {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = kGemmBM;   // 128 slices
constexpr int BN = 128;       // points
constexpr int BK = kGemmBK;   // 16
constexpr int LDA = BK + 4;   // padded LDS row (80 B): conflict-free 16-byte reads per 16 lanes

template <typename InT>
struct PointLoader {
  // Loads the BN x BK tile of union rows [l0, l0+BN) and columns [k0, k0+BK)
  // into registers (2 groups of 4 consecutive columns per thread).
  const InT *x, *y;
  int64_t N, M, L;
  int d;
  bool vec;   // d % 4 == 0 and FP32: one 16-byte load per group

  __device__ __forceinline__ void load(int64_t l0, int k0, float4 (&r)[2]) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = t + i * 256;          // 512 groups of 4 columns
      const int row = e >> 2, k4 = (e & 3) * 4;
      const int64_t l = l0 + row;
      const int k = k0 + k4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (l < L) {
        const InT *src = (l < M) ? (y + l * (int64_t)d) : (x + (l - M) * (int64_t)d);
        if constexpr (sizeof(InT) == 4) {
          if (vec) {
            if (k < d) v = *reinterpret_cast<const float4 *>(src + k);
          } else {
            if (k + 0 < d) v.x = (float)src[k + 0];
            if (k + 1 < d) v.y = (float)src[k + 1];
            if (k + 2 < d) v.z = (float)src[k + 2];
            if (k + 3 < d) v.w = (float)src[k + 3];
          }
        } else {
          if (k + 0 < d) v.x = (float)src[k + 0];
          if (k + 1 < d) v.y = (float)src[k + 1];
          if (k + 2 < d) v.z = (float)src[k + 2];
          if (k + 3 < d) v.w = (float)src[k + 3];
        }
      }
      r[i] = v;
    }
  }
};

template <typename InT>
__global__ __launch_bounds__(256) void proj_gemm_kernel(const float *__restrict__ dirs, int d_pad,
                                                       int p0, int nsl, PointLoader<InT> ld,
                                                       float *__restrict__ Z, int64_t ldz,
                                                       uint32_t *__restrict__ bounds,
                                                       int n_col_tiles, int n_row_tiles) {
  __shared__ float As[2][BM * LDA];
  __shared__ float Bs[2][BN * LDA];

  const int64_t work = xcd_remap(blockIdx.x, (int64_t)n_col_tiles * n_row_tiles);
  if (work < 0) return;
  // the row tiles of one point tile are consecutive work items (same XCD, X read once)
  const int col_tile = (int)(work / n_row_tiles);
  const int row_tile = (int)(work % n_row_tiles);
  const int64_t l0 = (int64_t)col_tile * BN;
  const int r0 = row_tile * BM;                 // local slice row of the tile
  const float *A = dirs + (int64_t)(p0 + r0) * d_pad;

  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 31, lh = lane >> 5;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  auto load_a = [&](int k0, float4 (&r)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = t + i * 256;
      const int row = e >> 2, k4 = (e & 3) * 4;
      r[i] = *reinterpret_cast<const float4 *>(A + (int64_t)row * d_pad + k0 + k4);
    }
  };
  auto store_tile = [&](float *S, const float4 (&r)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = t + i * 256;
      const int row = e >> 2, k4 = (e & 3) * 4;
      *reinterpret_cast<float4 *>(S + row * LDA + k4) = r[i];
    }
  };

  float4 ra[2], rb[2];
  load_a(0, ra);
  ld.load(l0, 0, rb);
  store_tile(As[0], ra);
  store_tile(Bs[0], rb);
  __syncthreads();

  const int nk = d_pad / BK;
  for (int kb = 0; kb < nk; ++kb) {
    const int cur = kb & 1;
    const bool more = kb + 1 < nk;
    if (more) {
      load_a((kb + 1) * BK, ra);
      ld.load(l0, (kb + 1) * BK, rb);
    }
    float a[2][8], b[2][8];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float *pa = As[cur] + (wm * 64 + i * 32 + lr) * LDA + lh * 8;
      const float4 a0 = *reinterpret_cast<const float4 *>(pa);
      const float4 a1 = *reinterpret_cast<const float4 *>(pa + 4);
      a[i][0] = a0.x; a[i][1] = a0.y; a[i][2] = a0.z; a[i][3] = a0.w;
      a[i][4] = a1.x; a[i][5] = a1.y; a[i][6] = a1.z; a[i][7] = a1.w;
      const float *pb = Bs[cur] + (wn * 64 + i * 32 + lr) * LDA + lh * 8;
      const float4 b0 = *reinterpret_cast<const float4 *>(pb);
      const float4 b1 = *reinterpret_cast<const float4 *>(pb + 4);
      b[i][0] = b0.x; b[i][1] = b0.y; b[i][2] = b0.z; b[i][3] = b0.w;
      b[i][4] = b1.x; b[i][5] = b1.y; b[i][6] = b1.z; b[i][7] = b1.w;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    if (more) {
      store_tile(As[cur ^ 1], ra);
      store_tile(Bs[cur ^ 1], rb);
    }
    __syncthreads();
  }

  // Epilogue: store Z (slice-major) and reduce per-slice min / max.
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = r0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);   // local slice
      float vmin = __builtin_huge_valf(), vmax = -__builtin_huge_valf();
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t l = l0 + wn * 64 + j * 32 + lr;
        const float v = acc[i][j][r];
        if (row < nsl && l < ld.L) {
          Z[(int64_t)row * ldz + l] = v;
          vmin = fminf(vmin, v);
          vmax = fmaxf(vmax, v);
        }
      }
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        vmin = fminf(vmin, __shfl_xor(vmin, off, 64));
        vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
      }
      if (lr == 0 && row < nsl && vmin <= vmax) {
        atomicMin(bounds + 2 * row, float_key(vmin));
        atomicMax(bounds + 2 * row + 1, float_key(vmax));
      }
    }
  }
}

__global__ void bounds_init_kernel(uint32_t *bounds, int nsl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsl) {
    bounds[2 * i] = 0xffffffffu;
    bounds[2 * i + 1] = 0u;
  }
}

hipError_t launch_projection(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  uint32_t *bounds = wsp<uint32_t>(a, lay.off_bounds);
  float *Z = wsp<float>(a, lay.off_z);
  mark(a, ST_MISC);
  bounds_init_kernel<<<(a.nsl + 255) / 256, 256, 0, a.stream>>>(bounds, a.nsl);
  mark(a, ST_PROJECT);
  const int n_col = (int)((lay.L + BN - 1) / BN);
  const int n_row = (a.nsl + BM - 1) / BM;
  const int64_t grid = xcd_grid((int64_t)n_col * n_row);
  const float *dirs = pl.d_dirs;
  if (a.f64in) {
    PointLoader<double> ld{(const double *)a.x, (const double *)a.y, lay.N, lay.M, lay.L, pl.d, false};
    proj_gemm_kernel<double><<<(unsigned)grid, 256, 0, a.stream>>>(dirs, pl.d_pad, a.p0, a.nsl, ld, Z,
                                                                  lay.L, bounds, n_col, n_row);
  } else {
    const bool vec = (pl.d % 4 == 0) && ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.y % 16 == 0);
    PointLoader<float> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, pl.d, vec};
    proj_gemm_kernel<float><<<(unsigned)grid, 256, 0, a.stream>>>(dirs, pl.d_pad, a.p0, a.nsl, ld, Z,
                                                                 lay.L, bounds, n_col, n_row);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight preparation: deterministic FP64 sum of |w| (fixed-point scale of the
// sort path's prefix sums) and, for FP64 inputs, the FP32 copy of w.
// ---------------------------------------------------------------------------
template <typename WT>
__global__ __launch_bounds__(256) void wsum_partial_kernel(const WT *w, int64_t N, float *wf,
                                                           double *part) {
  __shared__ double sm[64];
  const int64_t chunk = (N + kWsumBlocks - 1) / kWsumBlocks;
  const int64_t b0 = blockIdx.x * chunk, b1 = min(N, b0 + chunk);
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const float v = (float)w[i];
    if (wf) wf[i] = v;
    acc += fabs((double)v);
  }
  double tot;
  block_exclusive_scan(acc, sm, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void wsum_final_kernel(const double *part, double *misc) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kWsumBlocks; ++i) s += part[i];
    misc[0] = s;
    // fixed-point exponent eA: 2^eA * sum|w| < 2^61
    int e = 0;
    if (s > 0.0) {
      frexp(s, &e);   // s < 2^e
      misc[1] = (double)(61 - e);
    } else {
      misc[1] = 0.0;
    }
  }
}

hipError_t launch_weight_prep(const ExecArgs &a, const double *w64) {
  const Layout &lay = *a.lay;
  double *part = wsp<double>(a, lay.off_wpart);
  double *misc = wsp<double>(a, lay.off_misc);
  mark(a, ST_MISC);
  if (w64) {
    float *wf = wsp<float>(a, lay.off_wf);
    wsum_partial_kernel<double><<<kWsumBlocks, 256, 0, a.stream>>>(w64, lay.N, wf, part);
  } else {
    wsum_partial_kernel<float><<<kWsumBlocks, 256, 0, a.stream>>>(a.w, lay.N, nullptr, part);
  }
  wsum_final_kernel<<<1, 64, 0, a.stream>>>(part, misc);
  return hipGetLastError();
}

}  // namespace ksum
