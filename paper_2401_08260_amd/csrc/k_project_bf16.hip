// Split-BF16 projection GEMM: the same Z = Xi [Y; X]^T with per-slice min / max as
// the FP32 kernel, on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16).
//
// Every FP32 operand a is split as a = a_hi + a_lo + r with a_hi = bf16(a) and
// a_lo = bf16(a - a_hi) (round to nearest even), |r| <= 2^-17 |a|, and a product is
// taken as a_hi b_hi + a_hi b_lo + a_lo b_hi.  Each bf16 x bf16 product is exact
// in FP32 and the sum is accumulated in FP32, so the dropped terms (a_lo b_lo and
// the residuals r) are about 2^-16 |a b|: the result is close to an FP32 dot
// product at a sixteenth of the FP32 MFMA cycles per product.
//
// The directions are split once when the plan is made; the points are split as
// their tile is moved from registers to LDS.  A workgroup computes 128 slices x
// 256 points (4 waves, 2 x 2, each 64 slices x 128 points = 2 x 4 MFMA blocks),
// K step 16 double buffered in LDS.  An LDS row holds the 16 hi values of the step
// (32 B), then the 16 lo values (32 B), padded to 80 B so that the 16-byte fragment
// reads of 8 neighbouring rows fall on distinct banks.  Lane l of an MFMA supplies
// row l % 32 and the 8 contraction indices 8 (l / 32) .. + 7 of the step for both
// operands.
#include <algorithm>

#include "project_common.h"

namespace ksum {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int SM = 128;          // slices per tile
constexpr int SN = 256;          // points per tile
constexpr int SK = kGemmBK;      // 16
constexpr int ROWB = 80;         // bytes per LDS row (32 hi + 32 lo + 16 pad)
constexpr int A_BYTES = SM * ROWB;
constexpr int B_BYTES = SN * ROWB;
constexpr int STAGE_BYTES = A_BYTES + B_BYTES;   // 30 KB
constexpr int LDC = SN + 4;      // floats per row of the staged output (32 rows at a time)

static_assert(32 * LDC * 4 <= 2 * STAGE_BYTES, "output staging must fit the stage buffers");

// hi / lo halves of 4 consecutive FP32 values, packed as 4 bf16 each
__device__ __forceinline__ void split4(const float4 v, uint2 &hi, uint2 &lo) {
  const bf16x2 h0 = {(__bf16)v.x, (__bf16)v.y};
  const bf16x2 h1 = {(__bf16)v.z, (__bf16)v.w};
  const bf16x2 l0 = {(__bf16)(v.x - (float)h0[0]), (__bf16)(v.y - (float)h0[1])};
  const bf16x2 l1 = {(__bf16)(v.z - (float)h1[0]), (__bf16)(v.w - (float)h1[1])};
  hi = make_uint2(__builtin_bit_cast(uint32_t, h0), __builtin_bit_cast(uint32_t, h1));
  lo = make_uint2(__builtin_bit_cast(uint32_t, l0), __builtin_bit_cast(uint32_t, l1));
}

}  // namespace

template <typename InT, int VW>
__global__ __launch_bounds__(256, 2) void proj_gemm_bf16x3_kernel(GemmCtl g, PointLoader<InT, VW> ld) {
  __shared__ __align__(16) char smem[2 * STAGE_BYTES];
  __shared__ uint32_t smin[kMaxBatch], smax[kMaxBatch];
  __shared__ int s_tile;

  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 31, lh = lane >> 5;
  for (int i = t; i < g.nsl; i += 256) {
    smin[i] = 0xffffffffu;
    smax[i] = 0u;
  }
  const int total = g.n_col_tiles * g.n_row_tiles;
  const int nk = g.d_pad / SK;
  auto As = [&](int b) { return smem + b * STAGE_BYTES; };
  auto Bs = [&](int b) { return smem + b * STAGE_BYTES + A_BYTES; };
  // direction tile: thread t moves 8 hi and 8 lo values of row t / 2
  const int arow = t >> 1, akh = (t & 1) * 8;

  while (true) {
    if (t == 0) s_tile = (int)atomicAdd(g.counter, 1u);
    __syncthreads();
    const int tile = s_tile;
    if (tile >= total) break;
    const int col_tile = tile / g.n_row_tiles;
    const int row_tile = tile % g.n_row_tiles;
    const int64_t l0 = (int64_t)col_tile * SN;
    const int r0 = row_tile * SM;
    const int64_t aoff = (int64_t)(g.p0 + r0 + arow) * g.d_pad + akh;

    f32x16 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    auto store_a = [&](char *S, uint4 hi, uint4 lo) {
      *reinterpret_cast<uint4 *>(S + arow * ROWB + akh * 2) = hi;
      *reinterpret_cast<uint4 *>(S + arow * ROWB + 32 + akh * 2) = lo;
    };
    auto store_b = [&](char *S, int e, float4 v) {
      const int row = e >> 2, k4 = (e & 3) * 4;
      uint2 hi, lo;
      split4(v, hi, lo);
      *reinterpret_cast<uint2 *>(S + row * ROWB + k4 * 2) = hi;
      *reinterpret_cast<uint2 *>(S + row * ROWB + 32 + k4 * 2) = lo;
    };

    uint4 ah = *reinterpret_cast<const uint4 *>(g.dirs_hi + aoff);
    uint4 al = *reinterpret_cast<const uint4 *>(g.dirs_lo + aoff);
    float4 b0 = ld.load1(l0, 0, t), b1 = ld.load1(l0, 0, t + 256);
    float4 b2 = ld.load1(l0, 0, t + 512), b3 = ld.load1(l0, 0, t + 768);
    store_a(As(0), ah, al);
    store_b(Bs(0), t, b0);
    store_b(Bs(0), t + 256, b1);
    store_b(Bs(0), t + 512, b2);
    store_b(Bs(0), t + 768, b3);
    __syncthreads();

    for (int kb = 0; kb < nk; ++kb) {
      const int cur = kb & 1;
      const bool more = kb + 1 < nk;
      if (more) {
        const int k0 = (kb + 1) * SK;
        ah = *reinterpret_cast<const uint4 *>(g.dirs_hi + aoff + k0);
        al = *reinterpret_cast<const uint4 *>(g.dirs_lo + aoff + k0);
        b0 = ld.load1(l0, k0, t);
        b1 = ld.load1(l0, k0, t + 256);
        b2 = ld.load1(l0, k0, t + 512);
        b3 = ld.load1(l0, k0, t + 768);
      }
      const char *pa = As(cur) + (wm * 64 + lr) * ROWB + lh * 16;
      const char *pb = Bs(cur) + (wn * 128 + lr) * ROWB + lh * 16;
      bf16x8 fa_hi[2], fa_lo[2], fb_hi[4], fb_lo[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa_hi[i] = *reinterpret_cast<const bf16x8 *>(pa + i * 32 * ROWB);
        fa_lo[i] = *reinterpret_cast<const bf16x8 *>(pa + i * 32 * ROWB + 32);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        fb_hi[j] = *reinterpret_cast<const bf16x8 *>(pb + j * 32 * ROWB);
        fb_lo[j] = *reinterpret_cast<const bf16x8 *>(pb + j * 32 * ROWB + 32);
      }
      // small terms first, then hi x hi
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_lo[i], fb_hi[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_hi[i], fb_lo[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_hi[i], fb_hi[j], acc[i][j], 0, 0, 0);
        }
      if (more) {
        store_a(As(cur ^ 1), ah, al);
        store_b(Bs(cur ^ 1), t, b0);
        store_b(Bs(cur ^ 1), t + 256, b1);
        store_b(Bs(cur ^ 1), t + 512, b2);
        store_b(Bs(cur ^ 1), t + 768, b3);
      }
      __syncthreads();
    }

    // Epilogue in four passes of 32 slices (h = slice half, i = MFMA row block): the
    // waves holding the rows stage them in LDS, then every thread takes 32 values of
    // one row (8 float4 at a stride of 32 columns: 8 neighbouring threads cover 128
    // contiguous bytes per store), writes them to Z and folds them into the row's
    // min / max.
    float *C = reinterpret_cast<float *>(smem);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (wm == h) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              C[(8 * (r >> 2) + 4 * lh + (r & 3)) * LDC + wn * 128 + j * 32 + lr] = acc[i][j][r];
        }
        __syncthreads();
        const int lrow = t >> 3;                           // row within the 32
        const int row = r0 + h * 64 + i * 32 + lrow;       // slice within the batch
        const int c0 = (t & 7) * 4;
        float vmin = __builtin_huge_valf(), vmax = -__builtin_huge_valf();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + 32 * k;
          const float4 v = *reinterpret_cast<const float4 *>(C + lrow * LDC + c);
          const int64_t l = l0 + c;
          if (row < g.nsl) {
            float *dst = g.Z + (int64_t)row * g.ldz + l;
            if (g.z_vec4 && l + 3 < ld.L) {
              store_z4(dst, v);
            } else {
              if (l + 0 < ld.L) dst[0] = v.x;
              if (l + 1 < ld.L) dst[1] = v.y;
              if (l + 2 < ld.L) dst[2] = v.z;
              if (l + 3 < ld.L) dst[3] = v.w;
            }
          }
          if (l + 3 < ld.L) {
            vmin = fminf(vmin, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
            vmax = fmaxf(vmax, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
          } else {
            if (l + 0 < ld.L) { vmin = fminf(vmin, v.x); vmax = fmaxf(vmax, v.x); }
            if (l + 1 < ld.L) { vmin = fminf(vmin, v.y); vmax = fmaxf(vmax, v.y); }
            if (l + 2 < ld.L) { vmin = fminf(vmin, v.z); vmax = fmaxf(vmax, v.z); }
          }
        }
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
          vmin = fminf(vmin, __shfl_xor(vmin, off, 64));
          vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
        }
        if ((t & 7) == 0 && row < g.nsl && vmin <= vmax) {
          atomicMin(&smin[row], float_key(vmin));
          atomicMax(&smax[row], float_key(vmax));
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  uint32_t *out = g.part + (int64_t)blockIdx.x * g.nsl * 2;
  for (int i = t; i < g.nsl; i += 256) {
    out[2 * i] = smin[i];
    out[2 * i + 1] = smax[i];
  }
}

int projection_bf16x3_blocks(int64_t L, int nsl) {
  const int64_t tiles = ((L + SN - 1) / SN) * (int64_t)((nsl + SM - 1) / SM);
  return (int)std::min<int64_t>(tiles, 256 * kGemmBlocksPerCU);
}

hipError_t launch_projection_bf16x3(const ExecArgs &a, GemmCtl g) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  g.n_col_tiles = (int)((lay.L + SN - 1) / SN);
  g.n_row_tiles = (a.nsl + SM - 1) / SM;
  const unsigned grid = (unsigned)projection_bf16x3_blocks(lay.L, a.nsl);
  const int d = pl.d;
  const bool al16 = ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.y % 16 == 0);
  const bool al8 = ((uintptr_t)a.x % 8 == 0) && ((uintptr_t)a.y % 8 == 0);
  if (a.f64in) {
    PointLoader<double, 1> ld{(const double *)a.x, (const double *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<double, 1><<<grid, 256, 0, a.stream>>>(g, ld);
  } else if (d % 4 == 0 && al16) {
    PointLoader<float, 4> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<float, 4><<<grid, 256, 0, a.stream>>>(g, ld);
  } else if (d % 2 == 0 && al8) {
    PointLoader<float, 2> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<float, 2><<<grid, 256, 0, a.stream>>>(g, ld);
  } else {
    PointLoader<float, 1> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<float, 1><<<grid, 256, 0, a.stream>>>(g, ld);
  }
  return hipGetLastError();
}

}  // namespace ksum
