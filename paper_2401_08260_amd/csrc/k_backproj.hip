// Back-projection of the backward pass: the gradient with respect to a point set is
//
//   out[r][i] = scale_r * factor * sum_p D[r][p] xi_p[i],
//
// the per-target derivative sums D (one row per point, one column per slice)
// times the directions, i.e. the chain rule through the projections <xi_p, u_r>
// of the first step of Algorithm "Sliced Fast Fourier Summation".  A plain NT GEMM
// on the FP32 matrix cores (v_mfma_f32_32x32x2f32): tiles of 128 rows x 128
// dimensions per workgroup (4 waves, 2 x 2, each 64 x 64 = 2 x 2 MFMA blocks), the
// slice index as the contraction, K step 16 double buffered in LDS.  D and the
// transposed directions are zero beyond P, so the padded K steps add nothing.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace ksum {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TB = 128;          // rows and columns of a tile
constexpr int BK = kGemmBK;      // 16
constexpr int LDA = BK + 4;      // padded LDS row (80 B)
constexpr int LDC = TB + 4;

struct BackArgs {
  const float *D;        // [R][ldd]
  int64_t ldd;
  const float *dirsT;    // [d][Pk]
  int Pk, d;
  int64_t R;
  const float *scale;    // [R]
  float factor;
  float *out;            // [R][d]
  int out_vec4;          // rows of out are 16-byte aligned (d % 4 == 0, out 16-byte aligned)
};

// 4 consecutive values of row `row` at column k of a [rows][ld] matrix (zero outside)
__device__ __forceinline__ float4 load_row4(const float *base, int64_t ld, int64_t row, int64_t rows, int k) {
  if (row >= rows) return make_float4(0.f, 0.f, 0.f, 0.f);
  return *reinterpret_cast<const float4 *>(base + row * ld + k);
}

}  // namespace

__global__ __launch_bounds__(256) void backproject_kernel(BackArgs g) {
  __shared__ __align__(16) float smem[2 * 2 * TB * LDA];
  auto As = [&](int b) { return smem + b * (TB * LDA); };
  auto Bs = [&](int b) { return smem + 2 * TB * LDA + b * (TB * LDA); };
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 31, lh = lane >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * TB;
  const int c0 = blockIdx.y * TB;
  const int nk = g.Pk / BK;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // element e of the 512 float4 of a 128 x 16 tile: row e / 4, columns 4 (e % 4) .. + 3
  auto ldA = [&](int k0, int e) { return load_row4(g.D, g.ldd, r0 + (e >> 2), g.R, k0 + (e & 3) * 4); };
  auto ldB = [&](int k0, int e) { return load_row4(g.dirsT, g.Pk, c0 + (e >> 2), g.d, k0 + (e & 3) * 4); };
  auto st4 = [&](float *S, int e, float4 v) {
    *reinterpret_cast<float4 *>(S + (e >> 2) * LDA + (e & 3) * 4) = v;
  };

  // fragments of one half of a lane's 8 contraction indices (its first or last 4) in buffer b
  auto frag = [&](int b, int half, float4 (&fa)[2], float4 (&fb)[2]) {
    const float *pa = As(b) + (wm * 64 + lr) * LDA + lh * 8 + half * 4;
    const float *pb = Bs(b) + (wn * 64 + lr) * LDA + lh * 8 + half * 4;
    fa[0] = *reinterpret_cast<const float4 *>(pa);
    fa[1] = *reinterpret_cast<const float4 *>(pa + 32 * LDA);
    fb[0] = *reinterpret_cast<const float4 *>(pb);
    fb[1] = *reinterpret_cast<const float4 *>(pb + 32 * LDA);
  };
  auto mfma_half = [&](const float4 (&fa)[2], const float4 (&fb)[2]) {
    const float av[2][4] = {{fa[0].x, fa[0].y, fa[0].z, fa[0].w}, {fa[1].x, fa[1].y, fa[1].z, fa[1].w}};
    const float bv[2][4] = {{fb[0].x, fb[0].y, fb[0].z, fb[0].w}, {fb[1].x, fb[1].y, fb[1].z, fb[1].w}};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
  };

  float4 ra0 = ldA(0, t), ra1 = ldA(0, t + 256);
  float4 rb0 = ldB(0, t), rb1 = ldB(0, t + 256);
  st4(As(0), t, ra0);
  st4(As(0), t + 256, ra1);
  st4(Bs(0), t, rb0);
  st4(Bs(0), t + 256, rb1);
  __syncthreads();
  if (nk > 1) {
    ra0 = ldA(BK, t);
    ra1 = ldA(BK, t + 256);
    rb0 = ldB(BK, t);
    rb1 = ldB(BK, t + 256);
  }
  float4 flo_a[2], flo_b[2], fhi_a[2], fhi_b[2];
  frag(0, 0, flo_a, flo_b);
  // software pipeline over the K-blocks (as in the projection GEMM): the second half's
  // fragments are read during the first half's MFMAs, and after the barrier the next
  // block's first-half reads overlap the second half's MFMAs
  for (int kb = 0; kb < nk; ++kb) {
    const int cur = kb & 1;
    frag(cur, 1, fhi_a, fhi_b);
    __builtin_amdgcn_sched_barrier(0);
    mfma_half(flo_a, flo_b);
    __builtin_amdgcn_sched_barrier(0);
    if (kb + 1 < nk) {
      st4(As(cur ^ 1), t, ra0);
      st4(As(cur ^ 1), t + 256, ra1);
      st4(Bs(cur ^ 1), t, rb0);
      st4(Bs(cur ^ 1), t + 256, rb1);
    }
    __syncthreads();   // block kb + 1 stored; every wave's reads of buffer cur done
    if (kb + 2 < nk) {
      ra0 = ldA((kb + 2) * BK, t);
      ra1 = ldA((kb + 2) * BK, t + 256);
      rb0 = ldB((kb + 2) * BK, t);
      rb1 = ldB((kb + 2) * BK, t + 256);
    }
    if (kb + 1 < nk) frag(cur ^ 1, 0, flo_a, flo_b);
    __builtin_amdgcn_sched_barrier(0);
    mfma_half(fhi_a, fhi_b);
    __builtin_amdgcn_sched_barrier(0);
  }

  // epilogue in two halves of 64 rows through LDS: each thread writes 16 values of a row
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wm == h) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            smem[(i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3)) * LDC + wn * 64 + j * 32 + lr] = acc[i][j][r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int lrow = q * 32 + (t >> 3);
      const int64_t row = r0 + h * 64 + lrow;
      if (row < g.R) {
        const float sc = g.scale[row] * g.factor;
        float *dst = g.out + row * g.d;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = (t & 7) * 4 + 32 * k;
          const float4 v = *reinterpret_cast<const float4 *>(smem + lrow * LDC + c);
          if (g.out_vec4 && c0 + c + 3 < g.d) {
            // 16-byte non-temporal store: the gradient is far larger than the caches
            typedef float nt4 __attribute__((ext_vector_type(4)));
            const nt4 nv = {sc * v.x, sc * v.y, sc * v.z, sc * v.w};
            __builtin_nontemporal_store(nv, reinterpret_cast<nt4 *>(dst + c0 + c));
          } else {
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (c0 + c + u < g.d) dst[c0 + c + u] = sc * vv[u];
          }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_backproject(const ksum_plan &plan, const float *D, int64_t ldd, int64_t R, const float *scale,
                              double factor, float *out, hipStream_t stream) {
  BackArgs g{};
  g.D = D;
  g.ldd = ldd;
  g.dirsT = plan.d_dirsT;
  g.Pk = plan.Pk;
  g.d = plan.d;
  g.R = R;
  g.scale = scale;
  g.factor = (float)factor;
  g.out = out;
  g.out_vec4 = (plan.d % 4 == 0 && (uintptr_t)out % 16 == 0) ? 1 : 0;
  dim3 grid((unsigned)((R + TB - 1) / TB), (unsigned)((plan.d + TB - 1) / TB));
  backproject_kernel<<<grid, 256, 0, stream>>>(g);
  return hipGetLastError();
}

}  // namespace ksum
