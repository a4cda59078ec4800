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
// The directions are split once when the plan is made.  Plans with more than 8 tiles
// of 256 slices also split the points once per call (split_points_kernel), into a
// step-tiled layout that the kernel at the end of this file copies straight into
// LDS; otherwise the points are split as their tile moves from registers to LDS.  A workgroup of 8 waves computes 256
// slices x 256 points (waves 4 x 2, each 64 slices x 128 points = 2 x 4 MFMA
// blocks), one block per CU and so two waves per SIMD.  The K loop runs in steps
// of 32 (two MFMA contraction steps of 16, 48 MFMAs per wave between barriers)
// through two LDS stages: the global loads of step k + 1 are issued before step k
// is computed and go to the other stage after it, behind one barrier per step.  An
// LDS row holds the 32 hi values of the step (64 B), then the 32 lo values (64 B),
// padded to 144 B so that the 16-byte fragment reads of 8 neighbouring rows fall
// on distinct banks.  Lane l of an MFMA supplies row l % 32 and the 8 contraction
// indices 8 (l / 32) .. + 7 of its contraction step for both operands.
//
// Work items are (slice tile, point tile) pairs in slice-tile-major order, cut
// into 8 contiguous ranges, one per XCD (blocks are dispatched round-robin over
// the XCDs, so block b runs on XCD b % 8); the blocks of an XCD take the items of
// its range from their own counter.  An XCD so works on one slice tile at a time,
// whose directions (hi + lo) stay in its L2 while the point tiles stream past, and
// the XCDs that share a slice tile stream their point tiles in the same order.
#include <algorithm>

#include "project_common.h"

namespace ksum {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int NT = 512;          // threads per block
constexpr int SM = 256;          // slices per tile
constexpr int SN = 256;          // points per tile
constexpr int SK = 2 * kGemmBK;  // 32 (the plan pads d to it)
constexpr int ROWB = 144;        // bytes per LDS row (64 hi + 64 lo + 16 pad)
constexpr int A_BYTES = SM * ROWB;
constexpr int B_BYTES = SN * ROWB;
constexpr int STAGE_BYTES = A_BYTES + B_BYTES;   // 72 KB
constexpr int NSTAGE = 2;
constexpr int XCDS = 8;

static_assert(kGemmBM * 2 == SM, "the plan pads P to whole tiles of this kernel");

// hi / lo halves of 4 consecutive FP32 values, packed as 4 bf16 each
__device__ __forceinline__ void split4(const float4 v, uint2 &hi, uint2 &lo) {
  const bf16x2 h0 = {(__bf16)v.x, (__bf16)v.y};
  const bf16x2 h1 = {(__bf16)v.z, (__bf16)v.w};
  const bf16x2 l0 = {(__bf16)(v.x - (float)h0[0]), (__bf16)(v.y - (float)h0[1])};
  const bf16x2 l1 = {(__bf16)(v.z - (float)h1[0]), (__bf16)(v.w - (float)h1[1])};
  hi = make_uint2(__builtin_bit_cast(uint32_t, h0), __builtin_bit_cast(uint32_t, h1));
  lo = make_uint2(__builtin_bit_cast(uint32_t, l0), __builtin_bit_cast(uint32_t, l1));
}

// 4 consecutive values of a point row from column k (zero at and beyond d for VW < 4).
// The 16-byte path (VW = 4, d % 4 == 0) loads from a column clamped into the row; the
// values past d are set to zero when the step is stored (zero_tail), not here, so
// that nothing waits for the load before it is needed.  Rows beyond the union were
// pointed at a valid row by the caller (their products go to columns that are never
// stored).
template <typename InT, int VW>
__device__ __forceinline__ float4 row4(const InT *src, int k, int d) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (VW == 4) {
    v = *reinterpret_cast<const float4 *>(src + min(k, d - 4));
  } else if constexpr (VW == 2) {
    if (k < d) {
      const float2 q = *reinterpret_cast<const float2 *>(src + k);
      v.x = q.x;
      v.y = q.y;
    }
    if (k + 2 < d) {
      const float2 q = *reinterpret_cast<const float2 *>(src + k + 2);
      v.z = q.x;
      v.w = q.y;
    }
  } else {
    if (k + 0 < d) v.x = (float)src[k + 0];
    if (k + 1 < d) v.y = (float)src[k + 1];
    if (k + 2 < d) v.z = (float)src[k + 2];
    if (k + 3 < d) v.w = (float)src[k + 3];
  }
  return v;
}

__device__ __forceinline__ float4 zero_tail(float4 v, bool in) {
  return make_float4(in ? v.x : 0.f, in ? v.y : 0.f, in ? v.z : 0.f, in ? v.w : 0.f);
}

// The global data of one K step held by a thread between its load and its LDS store:
// 16 hi and 16 lo direction values of one row, and 4 x 4 point values.
struct StepRegs {
  uint4 ah0, ah1, al0, al1;
  float4 b[4];
};

}  // namespace

// Splits the union's points once into the step-tiled layout (tile_swz): hi = bf16(u_l[k]),
// lo = bf16(u_l[k] - hi) for rows l < rows and k < d_pad (zero for l >= L or k >= d).
// Thread e takes 16 values (one step) of one row and writes their 64 bytes: 16
// consecutive threads take 16 consecutive rows at one step and groups of 16 take
// consecutive steps, so a wave reads 256 consecutive bytes of each of 16 rows and
// writes 1 KB blocks.  rows is a multiple of 16.
template <typename InT, int VW>
__global__ __launch_bounds__(256) void split_points_kernel(const InT *x, const InT *y, int64_t M, int64_t L,
                                                          int d, int nst, int64_t rows, uint16_t *out) {
  const int64_t n = rows * nst;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t grp = e / (16 * nst);
    const int rem = (int)(e - grp * 16 * nst);
    const int64_t l = grp * 16 + (rem & 15);
    const int s = rem >> 4;
    const int k0 = s * 16;
    const InT *src = (l < M) ? y + l * (int64_t)d : x + (l - M) * (int64_t)d;
    uint2 h[4], lo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * q;
      // 4 values from column k (zero past d for VW < 4; VW = 4 means d % 4 == 0)
      const float4 v = (l < L && k < d) ? row4<InT, VW>(src, k, d) : make_float4(0.f, 0.f, 0.f, 0.f);
      split4(v, h[q], lo[q]);
    }
    const uint4 chunk[4] = {make_uint4(h[0].x, h[0].y, h[1].x, h[1].y), make_uint4(h[2].x, h[2].y, h[3].x, h[3].y),
                            make_uint4(lo[0].x, lo[0].y, lo[1].x, lo[1].y),
                            make_uint4(lo[2].x, lo[2].y, lo[3].x, lo[3].y)};
    uint4 *dst = reinterpret_cast<uint4 *>(out + ((int64_t)s * rows + l) * 32);
    const int sw = tile_swz(l);
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[c ^ sw] = chunk[c];
  }
}

template <typename InT, int VW>
__global__ __launch_bounds__(NT, 1) void proj_gemm_bf16x3_kernel(GemmCtl g, PointLoader<InT, VW> ld) {
  __shared__ __align__(16) char smem[NSTAGE * STAGE_BYTES];
  __shared__ uint32_t smin[kMaxBatch], smax[kMaxBatch];
  __shared__ int s_item;

  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 1, wn = wid & 1;    // 64-slice rows wm, 128-point columns wn
  const int lr = lane & 31, lh = lane >> 5;
  for (int i = t; i < g.nsl; i += NT) {
    smin[i] = 0xffffffffu;
    smax[i] = 0u;
  }
  const int64_t total = (int64_t)g.n_col_tiles * g.n_row_tiles;
  const int xcd = blockIdx.x % XCDS;
  const int64_t lo = total * xcd / XCDS, hi = total * (xcd + 1) / XCDS;
  const int nk = g.d_pad / SK;
  const int d = ld.d;
  auto As = [&](int s) { return smem + s * STAGE_BYTES; };
  auto Bs = [&](int s) { return smem + s * STAGE_BYTES + A_BYTES; };
  // direction tile: thread t moves 16 hi and 16 lo values of row t / 2; point tile:
  // columns k4 .. k4 + 3 of rows t / 8 + 64 q, q = 0..3
  const int arow = t >> 1, akh = (t & 1) * 16;
  const int brow = t >> 3, k4 = (t & 7) * 4;

  while (true) {
    if (t == 0) s_item = (int)(lo + (int64_t)atomicAdd(g.counter + xcd, 1u));
    __syncthreads();
    const int64_t item = s_item;
    if (item >= hi) break;
    const int row_tile = (int)(item / g.n_col_tiles);
    const int64_t col_tile = item % g.n_col_tiles;
    const int64_t l0 = col_tile * SN;
    const int r0 = row_tile * SM;
    const int64_t aoff = (int64_t)(g.p0 + r0 + arow) * g.d_pad + akh;
    const uint16_t *ahp = g.dirs_hi + aoff;
    const uint16_t *alp = g.dirs_lo + aoff;
    const InT *bsrc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t l = l0 + brow + 64 * q;    // rows beyond the union read row 0 of y
      bsrc[q] = (l >= ld.L) ? ld.y : (l < ld.M) ? ld.y + l * (int64_t)d : ld.x + (l - ld.M) * (int64_t)d;
    }

    f32x16 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // steps past the end load the last step again (in bounds, never stored)
    auto load_step = [&](int kb) {
      const int k0 = min(kb, nk - 1) * SK;
      StepRegs R;
      R.ah0 = *reinterpret_cast<const uint4 *>(ahp + k0);
      R.ah1 = *reinterpret_cast<const uint4 *>(ahp + k0 + 8);
      R.al0 = *reinterpret_cast<const uint4 *>(alp + k0);
      R.al1 = *reinterpret_cast<const uint4 *>(alp + k0 + 8);
#pragma unroll
      for (int q = 0; q < 4; ++q) R.b[q] = row4<InT, VW>(bsrc[q], k0 + k4, d);
      return R;
    };
    auto store_step = [&](int s, int kb, const StepRegs &R) {
      char *A = As(s) + arow * ROWB + akh * 2;
      *reinterpret_cast<uint4 *>(A) = R.ah0;
      *reinterpret_cast<uint4 *>(A + 16) = R.ah1;
      *reinterpret_cast<uint4 *>(A + 64) = R.al0;
      *reinterpret_cast<uint4 *>(A + 80) = R.al1;
      const bool in = VW < 4 || kb * SK + k4 < d;
      char *B = Bs(s) + k4 * 2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint2 bh, bl;
        split4(zero_tail(R.b[q], in), bh, bl);
        char *p = B + (brow + 64 * q) * ROWB;
        *reinterpret_cast<uint2 *>(p) = bh;
        *reinterpret_cast<uint2 *>(p + 64) = bl;
      }
    };
    auto compute = [&](int s) {
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        const char *pa = As(s) + (wm * 64 + lr) * ROWB + sub * 32 + lh * 16;
        const char *pb = Bs(s) + (wn * 128 + lr) * ROWB + sub * 32 + lh * 16;
        bf16x8 fa_hi[2], fa_lo[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          fa_hi[i] = *reinterpret_cast<const bf16x8 *>(pa + i * 32 * ROWB);
          fa_lo[i] = *reinterpret_cast<const bf16x8 *>(pa + i * 32 * ROWB + 64);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bf16x8 fb_hi = *reinterpret_cast<const bf16x8 *>(pb + j * 32 * ROWB);
          const bf16x8 fb_lo = *reinterpret_cast<const bf16x8 *>(pb + j * 32 * ROWB + 64);
          // small terms first, then hi x hi
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_lo[i], fb_hi, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_hi[i], fb_lo, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_hi[i], fb_hi, acc[i][j], 0, 0, 0);
          }
        }
      }
    };

    // step kb: the loads of kb + 1 go out first, kb is computed from its stage, then
    // kb + 1 goes to the other stage (read during step kb - 1, before the last barrier)
    store_step(0, 0, load_step(0));
    __syncthreads();
    int s0 = 0;
    for (int kb = 0; kb < nk; ++kb) {
      const StepRegs R = load_step(kb + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(s0);
      __builtin_amdgcn_sched_barrier(0);
      if (kb + 1 < nk) store_step(s0 ^ 1, kb + 1, R);
      __syncthreads();
      s0 ^= 1;
    }

    // Epilogue straight from the accumulators: element r of block (i, j) of a lane is
    // slice row wm * 64 + 32 i + 8 (r / 4) + 4 lh + r % 4 and point column
    // wn * 128 + 32 j + lr, so one store instruction covers two rows of 32 consecutive
    // points (two 128-byte runs).  Row minima / maxima: over the lane's 4 point blocks,
    // then over the 32 lanes of the row, then into LDS.
    const int64_t cbase = l0 + wn * 128 + lr;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = r0 + wm * 64 + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
        float vmin = __builtin_huge_valf(), vmax = -__builtin_huge_valf();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t l = cbase + 32 * j;
          const float v = acc[i][j][r];
          if (l < ld.L) {
            if (row < g.nsl) __builtin_nontemporal_store(v, g.Z + (int64_t)row * g.ldz + l);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
          }
        }
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) {
          vmin = fminf(vmin, __shfl_xor(vmin, off, 64));
          vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
        }
        if (lr == 0 && row < g.nsl && vmin <= vmax) {
          atomicMin(&smin[row], float_key(vmin));
          atomicMax(&smax[row], float_key(vmax));
        }
      }
    }
  }
  __syncthreads();
  uint32_t *out = g.part + (int64_t)blockIdx.x * g.nsl * 2;
  for (int i = t; i < g.nsl; i += NT) {
    out[2 * i] = smin[i];
    out[2 * i + 1] = smax[i];
  }
}

// ---------------------------------------------------------------------------
// Step-tiled operands (pre-split points): a K step of a 256-row tile of either
// operand is one contiguous 16 KB block in global memory, laid out as it is needed in
// LDS, so it goes straight into LDS (global_load_lds_dwordx4: each lane's 16 bytes
// land at the wave's LDS address + 16 x lane) without passing through registers;
// every copy instruction moves 1 KB of consecutive bytes.  Steps of 16 contraction
// indices, four LDS stages of 32 KB, copies issued three steps ahead; one barrier per
// step, before which every wave waits only for its own copies of the step about to
// be read.
//
// An LDS row is 64 bytes: 16-byte chunks c = 0, 1 (hi, k 0..7 and 8..15) and 2, 3
// (lo), chunk c of global row r in slot c ^ tile_swz(r).  The fragment reads of 8 (or
// 16) consecutive rows at one chunk then hit distinct bank groups whether the LDS
// serves 128 or 256 bytes per cycle.
//
// The compiler is not told about these copies (they are written as inline asm):
// it would otherwise wait for all of them before every LDS read.  The waits are
// explicit vmcnt counts; every other memory operation of the K loop is an LDS read.
// ---------------------------------------------------------------------------
namespace {

constexpr int DK = kGemmBK;             // contraction indices per step (16)
constexpr int DROW = DK * 4;            // bytes per LDS row: 32 hi + 32 lo
constexpr int DTILE = SM * DROW;        // 16 KB per operand tile
constexpr int DSTAGE = 2 * DTILE;       // A tile, then B tile
constexpr int DNS = 4;                  // stages
static_assert(SM == SN, "one row layout for both operands");

// The 4 copies of one step of one wave: A rows (2 x 16) and B rows (2 x 16).
__device__ __forceinline__ void dma_step(const char *a0, const char *a1, const char *b0, const char *b1,
                                         uint32_t la0, uint32_t la1, uint32_t lb0, uint32_t lb1) {
  asm volatile(
      "s_mov_b32 m0, %4\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off\n\t"
      "s_mov_b32 m0, %5\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off\n\t"
      "s_mov_b32 m0, %6\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %7\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %3, off"
      :
      : "v"(a0), "v"(a1), "v"(b0), "v"(b1), "s"(la0), "s"(la1), "s"(lb0), "s"(lb1)
      : "memory", "m0");
}

// s_waitcnt with only the vector-memory count set (expcnt and lgkmcnt at their maxima)
template <int N> __device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt field");
  __builtin_amdgcn_s_waitcnt(N | (0x7 << 4) | (0xF << 8));
}

}  // namespace

__global__ __launch_bounds__(NT, 1) void proj_gemm_bf16x3_dma_kernel(GemmCtl g, int64_t L) {
  __shared__ __align__(1024) char smem[DNS * DSTAGE];
  __shared__ uint32_t smin[kMaxBatch], smax[kMaxBatch];
  __shared__ int s_item;

  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 31, lh = lane >> 5;
  const uint32_t wu = __builtin_amdgcn_readfirstlane(wid);
  for (int i = t; i < g.nsl; i += NT) {
    smin[i] = 0xffffffffu;
    smax[i] = 0u;
  }
  const int64_t total = (int64_t)g.n_col_tiles * g.n_row_tiles;
  const int xcd = blockIdx.x % XCDS;
  const int64_t lo = total * xcd / XCDS, hi = total * (xcd + 1) / XCDS;
  const int nk = g.d_pad / DK;
  const uint32_t lds0 = (uint32_t)(uintptr_t)smem;
  // fragment reads of the point tile: tile row R = wn * 128 + 32 j + lr is global row
  // l0 + R with l0 a multiple of 256, and tile_swz only looks at bits 1..4, so the slot
  // of its chunk c is c ^ tile_swz(lr)
  const int fswb = tile_swz(lr);
  const int offb_hi = lr * DROW + ((lh ^ fswb) << 4), offb_lo = lr * DROW + (((2 + lh) ^ fswb) << 4);

  while (true) {
    if (t == 0) s_item = (int)(lo + (int64_t)atomicAdd(g.counter + xcd, 1u));
    __syncthreads();
    const int64_t item = s_item;
    if (item >= hi) break;
    const int row_tile = (int)(item / g.n_col_tiles);
    const int64_t col_tile = item % g.n_col_tiles;
    const int64_t l0 = col_tile * SN;
    const int r0 = row_tile * SM;
    // the slice tile starts at global row p0 + r0, which need not be a multiple of 32
    const int fswa = tile_swz(g.p0 + r0 + lr);
    const int offa_hi = lr * DROW + ((lh ^ fswa) << 4), offa_lo = lr * DROW + (((2 + lh) ^ fswa) << 4);
    // wave w copies bytes [2048 w, 2048 w + 2048) of the step's A and B blocks
    const char *ca = reinterpret_cast<const char *>(g.dirs_t + (int64_t)(g.p0 + r0) * 32) + wid * 2048 + lane * 16;
    const char *cb = reinterpret_cast<const char *>(g.pts_t + l0 * 32) + wid * 2048 + lane * 16;
    const int64_t astep = g.a_rows * DROW, bstep = g.b_rows * DROW;   // bytes per step
    auto issue = [&](int kb) {
      const uint32_t la = lds0 + (uint32_t)((kb & (DNS - 1)) * DSTAGE) + wu * 2048;
      const char *pa = ca + kb * astep, *pb = cb + kb * bstep;
      dma_step(pa, pa + 1024, pb, pb + 1024, la, la + 1024, la + DTILE, la + DTILE + 1024);
    };

    f32x16 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

#pragma unroll
    for (int s = 0; s < DNS - 1; ++s)
      if (s < nk) issue(s);
    for (int kb = 0; kb < nk; ++kb) {
      // this wave's copies of step kb are done once at most those of the (up to two)
      // later steps already issued are outstanding
      const int later = min(DNS - 2, nk - 1 - kb);
      if (later >= 2) wait_vm<8>();
      else if (later == 1) wait_vm<4>();
      else wait_vm<0>();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      // every wave is past step kb - 1, so its stage takes the copies of step kb + 3
      if (kb + DNS - 1 < nk) issue(kb + DNS - 1);
      const char *A = smem + (kb & (DNS - 1)) * DSTAGE;
      const char *B = A + DTILE;
      bf16x8 fa_hi[2], fa_lo[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const char *pa = A + (wm * 64 + i * 32) * DROW;
        fa_hi[i] = *reinterpret_cast<const bf16x8 *>(pa + offa_hi);
        fa_lo[i] = *reinterpret_cast<const bf16x8 *>(pa + offa_lo);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const char *pb = B + (wn * 128 + j * 32) * DROW;
        const bf16x8 fb_hi = *reinterpret_cast<const bf16x8 *>(pb + offb_hi);
        const bf16x8 fb_lo = *reinterpret_cast<const bf16x8 *>(pb + offb_lo);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_lo[i], fb_hi, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_hi[i], fb_lo, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa_hi[i], fb_hi, acc[i][j], 0, 0, 0);
        }
      }
    }

    // epilogue as in the kernel above
    const int64_t cbase = l0 + wn * 128 + lr;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = r0 + wm * 64 + 32 * i + 8 * (r >> 2) + 4 * lh + (r & 3);
        float vmin = __builtin_huge_valf(), vmax = -__builtin_huge_valf();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t l = cbase + 32 * j;
          const float v = acc[i][j][r];
          if (l < L) {
            if (row < g.nsl) __builtin_nontemporal_store(v, g.Z + (int64_t)row * g.ldz + l);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
          }
        }
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) {
          vmin = fminf(vmin, __shfl_xor(vmin, off, 64));
          vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
        }
        if (lr == 0 && row < g.nsl && vmin <= vmax) {
          atomicMin(&smin[row], float_key(vmin));
          atomicMax(&smax[row], float_key(vmax));
        }
      }
    }
  }
  __syncthreads();
  uint32_t *out = g.part + (int64_t)blockIdx.x * g.nsl * 2;
  for (int i = t; i < g.nsl; i += NT) {
    out[2 * i] = smin[i];
    out[2 * i + 1] = smax[i];
  }
}

// One block per CU, a multiple of 8 blocks so that every XCD's range has blocks.
int projection_bf16x3_blocks(int64_t L, int nsl) {
  const int64_t tiles = ((L + SN - 1) / SN) * (int64_t)((nsl + SM - 1) / SM);
  return (int)std::min<int64_t>(xcd_grid(tiles), 256);
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
  if (g.pts_t) {
    proj_gemm_bf16x3_dma_kernel<<<grid, NT, 0, a.stream>>>(g, lay.L);
  } else if (a.f64in) {
    PointLoader<double, 1> ld{(const double *)a.x, (const double *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<double, 1><<<grid, NT, 0, a.stream>>>(g, ld);
  } else if (d % 4 == 0 && al16) {
    PointLoader<float, 4> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<float, 4><<<grid, NT, 0, a.stream>>>(g, ld);
  } else if (d % 2 == 0 && al8) {
    PointLoader<float, 2> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<float, 2><<<grid, NT, 0, a.stream>>>(g, ld);
  } else {
    PointLoader<float, 1> ld{(const float *)a.x, (const float *)a.y, lay.N, lay.M, lay.L, d};
    proj_gemm_bf16x3_kernel<float, 1><<<grid, NT, 0, a.stream>>>(g, ld);
  }
  return hipGetLastError();
}

hipError_t launch_split_points(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  uint16_t *out = wsp<uint16_t>(a, lay.off_split);
  const int nst = pl.d_pad / kGemmBK;
  const int64_t n = lay.split_rows * nst;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
  mark(a, ST_SPLIT_POINTS);
  const int d = pl.d;
  const bool al16 = ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.y % 16 == 0);
  const bool al8 = ((uintptr_t)a.x % 8 == 0) && ((uintptr_t)a.y % 8 == 0);
  if (a.f64in)
    split_points_kernel<double, 1><<<grid, 256, 0, a.stream>>>((const double *)a.x, (const double *)a.y, lay.M,
                                                               lay.L, d, nst, lay.split_rows, out);
  else if (d % 4 == 0 && al16)
    split_points_kernel<float, 4><<<grid, 256, 0, a.stream>>>((const float *)a.x, (const float *)a.y, lay.M, lay.L, d,
                                                              nst, lay.split_rows, out);
  else if (d % 2 == 0 && al8)
    split_points_kernel<float, 2><<<grid, 256, 0, a.stream>>>((const float *)a.x, (const float *)a.y, lay.M, lay.L, d,
                                                              nst, lay.split_rows, out);
  else
    split_points_kernel<float, 1><<<grid, 256, 0, a.stream>>>((const float *)a.x, (const float *)a.y, lay.M, lay.L, d,
                                                              nst, lay.split_rows, out);
  return hipGetLastError();
}

}  // namespace ksum
