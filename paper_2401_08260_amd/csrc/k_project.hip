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
#include <algorithm>

#include "project_common.h"

namespace ksum {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = kGemmBM;   // 128 slices
constexpr int BN = 128;       // points
constexpr int BK = kGemmBK;   // 16
constexpr int LDA = BK + 4;   // padded LDS row (80 B): conflict-free 16-byte reads per 16 lanes
constexpr int LDC = BN + 4;   // padded row of the staged output tile

// Epilogue of a 128 x 128 tile, in two halves of 64 slices: the waves holding the
// half write their accumulators to LDS, then every thread takes 16 values of one
// row (4 float4 at a stride of 32 columns, so 8 neighbouring threads cover 128
// contiguous bytes per store), writes them to Z and folds them into the row's
// min / max.  smem must hold 64 x LDC floats and be free.
__device__ __forceinline__ void tile_epilogue(const GemmCtl &g, const f32x16 (&acc)[2][2], float *smem,
                                              uint32_t *smin, uint32_t *smax, int r0, int64_t l0, int64_t L) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 31, lh = lane >> 5;
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
      const int lrow = q * 32 + (t >> 3);            // row within the half
      const int row = r0 + h * 64 + lrow;            // slice within the batch
      const int c0 = (t & 7) * 4;
      float vmin = __builtin_huge_valf(), vmax = -__builtin_huge_valf();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = c0 + 32 * k;
        const float4 v = *reinterpret_cast<const float4 *>(smem + lrow * LDC + c);
        const int64_t l = l0 + c;
        if (row < g.nsl) {
          float *dst = g.Z + (int64_t)row * g.ldz + l;
          if (g.z_vec4 && l + 3 < L) {
            store_z4(dst, v);
          } else {
            if (l + 0 < L) dst[0] = v.x;
            if (l + 1 < L) dst[1] = v.y;
            if (l + 2 < L) dst[2] = v.z;
            if (l + 3 < L) dst[3] = v.w;
          }
        }
        if (l + 3 < L) {
          vmin = fminf(vmin, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
          vmax = fmaxf(vmax, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
        } else {
          if (l + 0 < L) { vmin = fminf(vmin, v.x); vmax = fmaxf(vmax, v.x); }
          if (l + 1 < L) { vmin = fminf(vmin, v.y); vmax = fmaxf(vmax, v.y); }
          if (l + 2 < L) { vmin = fminf(vmin, v.z); vmax = fmaxf(vmax, v.z); }
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
    }
    __syncthreads();
  }
}

// Persistent blocks take (point tile, slice tile) work items from a device
// counter in order, so neighbouring items (the slice tiles of one point tile)
// run at the same time and every CU ends within about one tile of the others.
// Per-slice min / max are kept in LDS and written once per block; the set-up
// kernel reduces the blocks' partials (no global atomics on 2P addresses).
template <typename InT, int VW>
__global__ __launch_bounds__(256) void proj_gemm_kernel(GemmCtl g, PointLoader<InT, VW> ld) {
  // K-loop tiles As[2][BM][LDA], Bs[2][BN][LDA]; after the K loop the same memory
  // stages half of the output tile (64 rows of LDC floats) for the epilogue
  __shared__ __align__(16) float smem[2 * (BM + BN) * LDA];
  auto As = [&](int b) { return smem + b * (BM * LDA); };
  auto Bs = [&](int b) { return smem + 2 * BM * LDA + b * (BN * LDA); };
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
  const int nk = g.d_pad / BK;

  while (true) {
    if (t == 0) s_tile = (int)atomicAdd(g.counter, 1u);
    __syncthreads();
    const int tile = s_tile;
    if (tile >= total) break;
    const int col_tile = tile / g.n_row_tiles;
    const int row_tile = tile % g.n_row_tiles;
    const int64_t l0 = (int64_t)col_tile * BN;
    const int r0 = row_tile * BM;
    const float *A = g.dirs + (int64_t)(g.p0 + r0) * g.d_pad;

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // element e of the 512 float4 of a 128 x 16 tile: row e / 4, columns 4 (e % 4) .. + 3
    auto load_a = [&](int k0, int e) {
      const int row = e >> 2, k4 = (e & 3) * 4;
      return *reinterpret_cast<const float4 *>(A + (int64_t)row * g.d_pad + k0 + k4);
    };
    auto store4 = [&](float *S, int e, float4 v) {
      const int row = e >> 2, k4 = (e & 3) * 4;
      *reinterpret_cast<float4 *>(S + row * LDA + k4) = v;
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
    // the 16 MFMAs of one half: 4 contraction steps x 2 x 2 blocks of 32 x 32
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

    float4 ra0 = load_a(0, t), ra1 = load_a(0, t + 256);
    float4 rb0 = ld.load1(l0, 0, t), rb1 = ld.load1(l0, 0, t + 256);
    store4(As(0), t, ra0);
    store4(As(0), t + 256, ra1);
    store4(Bs(0), t, rb0);
    store4(Bs(0), t + 256, rb1);
    __syncthreads();
    if (nk > 1) {
      ra0 = load_a(BK, t);
      ra1 = load_a(BK, t + 256);
      rb0 = ld.load1(l0, BK, t);
      rb1 = ld.load1(l0, BK, t + 256);
    }
    float4 flo_a[2], flo_b[2], fhi_a[2], fhi_b[2];
    frag(0, 0, flo_a, flo_b);

    // Software pipeline over the K-blocks, so that no wave waits for LDS while
    // all waves of the CU read it at once: at the top of iteration kb the first
    // half's fragments of kb are in flight and the loads of K-block kb + 1 are in
    // registers.  The first half's MFMAs overlap the second half's reads; the
    // next block goes to the other buffer; after the barrier the next block's
    // first-half reads and loads two blocks ahead overlap the second half's MFMAs.
    for (int kb = 0; kb < nk; ++kb) {
      const int cur = kb & 1;
      frag(cur, 1, fhi_a, fhi_b);
      __builtin_amdgcn_sched_barrier(0);
      mfma_half(flo_a, flo_b);
      __builtin_amdgcn_sched_barrier(0);
      if (kb + 1 < nk) {
        store4(As(cur ^ 1), t, ra0);
        store4(As(cur ^ 1), t + 256, ra1);
        store4(Bs(cur ^ 1), t, rb0);
        store4(Bs(cur ^ 1), t + 256, rb1);
      }
      __syncthreads();   // block kb + 1 stored; every wave's reads of buffer cur done
      if (kb + 2 < nk) {
        ra0 = load_a((kb + 2) * BK, t);
        ra1 = load_a((kb + 2) * BK, t + 256);
        rb0 = ld.load1(l0, (kb + 2) * BK, t);
        rb1 = ld.load1(l0, (kb + 2) * BK, t + 256);
      }
      if (kb + 1 < nk) frag(cur ^ 1, 0, flo_a, flo_b);
      __builtin_amdgcn_sched_barrier(0);
      mfma_half(fhi_a, fhi_b);
      __builtin_amdgcn_sched_barrier(0);
    }
    tile_epilogue(g, acc, smem, smin, smax, r0, l0, ld.L);
  }
  __syncthreads();
  uint32_t *out = g.part + (int64_t)blockIdx.x * g.nsl * 2;
  for (int i = t; i < g.nsl; i += 256) {
    out[2 * i] = smin[i];
    out[2 * i + 1] = smax[i];
  }
}

// clears the tile queue heads (one per XCD for the split-BF16 kernel, the first for FP32)
__global__ void gemm_init_kernel(uint32_t *counter) {
  if (threadIdx.x < 16 && blockIdx.x == 0) counter[threadIdx.x] = 0u;
}

int projection_blocks(const ksum_plan &plan, int64_t L, int nsl) {
  if (plan.params.precision == KSUM_SPLIT_BF16) return projection_bf16x3_blocks(L, nsl);
  const int64_t tiles = ((L + BN - 1) / BN) * (int64_t)((nsl + BM - 1) / BM);
  return (int)std::min<int64_t>(tiles, 256 * kGemmBlocksPerCU);
}

hipError_t launch_projection(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  GemmCtl g;
  g.dirs = pl.d_dirs;
  g.d_pad = pl.d_pad;
  g.p0 = a.p0;
  g.nsl = a.nsl;
  g.Z = wsp<float>(a, lay.off_z);
  g.ldz = lay.L;
  g.counter = wsp<uint32_t>(a, lay.off_counter);
  g.part = wsp<uint32_t>(a, lay.off_bounds_part);
  g.n_col_tiles = (int)((lay.L + BN - 1) / BN);
  g.n_row_tiles = (a.nsl + BM - 1) / BM;
  g.z_vec4 = (lay.L % 4 == 0) ? 1 : 0;
  g.dirs_hi = pl.d_dirs_hi;
  g.dirs_lo = pl.d_dirs_lo;
  g.dirs_t = pl.d_dirs_tiled;
  g.pts_t = lay.presplit ? wsp<uint16_t>(a, lay.off_split) : nullptr;
  g.a_rows = pl.P_pad;
  g.b_rows = lay.split_rows;
  mark(a, ST_MISC);
  gemm_init_kernel<<<1, 64, 0, a.stream>>>(g.counter);
  mark(a, ST_PROJECT);
  if (pl.params.precision == KSUM_SPLIT_BF16) return launch_projection_bf16x3(a, g);
  const unsigned grid = (unsigned)projection_blocks(pl, lay.L, a.nsl);
  const int d = pl.d;
  const bool al16 = ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.y % 16 == 0);
  const bool al8 = ((uintptr_t)a.x % 8 == 0) && ((uintptr_t)a.y % 8 == 0);
  if (a.f64in) {
    PointLoader<double, 1> ld{(const double *)a.x, (const double *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_kernel<double, 1><<<grid, 256, 0, a.stream>>>(g, ld);
  } else if (d % 4 == 0 && al16) {
    PointLoader<float, 4> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_kernel<float, 4><<<grid, 256, 0, a.stream>>>(g, ld);
  } else if (d % 2 == 0 && al8) {
    PointLoader<float, 2> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_kernel<float, 2><<<grid, 256, 0, a.stream>>>(g, ld);
  } else {
    PointLoader<float, 1> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_kernel<float, 1><<<grid, 256, 0, a.stream>>>(g, ld);
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
