// Device helpers shared by the ksum kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ksum {

// Order-preserving map float -> uint32 (with -0 mapped to +0): a < b as floats
// iff key(a) < key(b); equal floats (including -0 == +0) give equal keys.
__device__ __forceinline__ uint32_t float_key(float f) {
  uint32_t u = __float_as_uint(f);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// XCD-aware block remap: workgroups are dispatched round-robin over the 8 XCDs,
// so linear block b runs on XCD b % 8.  Mapping b to work item
// (b % 8) * per_xcd + b / 8 gives every XCD a contiguous range of work items,
// which keeps neighbouring work (same slice / same point tile) in one L2.
// Returns -1 for the padding blocks of the last round.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t total) {
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t w = (b % 8) * per_xcd + b / 8;
  return w < total ? w : -1;
}

__host__ __device__ inline int64_t xcd_grid(int64_t total) { return ((total + 7) / 8) * 8; }

// ---------------------------------------------------------------------------
// Wave scans through DPP (no LDS round trips): Hillis-Steele inside each row of
// 16 lanes (row_shr 1, 2, 4, 8), then lane 15 of rows 0 and 2 into rows 1 and 3
// (row_bcast:15) and lane 31 into rows 2 and 3 (row_bcast:31).  Lanes whose DPP
// source is outside the row, and rows the row mask leaves out, read `fill`.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const uint32_t lo = dpp_u32<CTRL, ROWS>((uint32_t)v, 0u);
  const uint32_t hi = dpp_u32<CTRL, ROWS>((uint32_t)(v >> 32), 0u);
  return ((unsigned long long)hi << 32) | lo;
}

// inclusive prefix sum over the 64 lanes (integer: exact, wraps like the type)
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  v += dpp_u32<0x111, 0xf>(v, 0u);
  v += dpp_u32<0x112, 0xf>(v, 0u);
  v += dpp_u32<0x114, 0xf>(v, 0u);
  v += dpp_u32<0x118, 0xf>(v, 0u);
  v += dpp_u32<0x142, 0xa>(v, 0u);
  v += dpp_u32<0x143, 0xc>(v, 0u);
  return v;
}

__device__ __forceinline__ long long wave_incl_sum(long long v) {
  unsigned long long u = (unsigned long long)v;
  u += dpp_u64<0x111, 0xf>(u);
  u += dpp_u64<0x112, 0xf>(u);
  u += dpp_u64<0x114, 0xf>(u);
  u += dpp_u64<0x118, 0xf>(u);
  u += dpp_u64<0x142, 0xa>(u);
  u += dpp_u64<0x143, 0xc>(u);
  return (long long)u;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  return __longlong_as_double((long long)dpp_u64<CTRL, ROWS>((unsigned long long)__double_as_longlong(v)));
}

// FP64 inclusive prefix sum over the 64 lanes (fixed order of additions)
__device__ __forceinline__ double wave_incl_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);
  v += dpp_f64<0x112, 0xf>(v);
  v += dpp_f64<0x114, 0xf>(v);
  v += dpp_f64<0x118, 0xf>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  return v;
}

// minimum / maximum over the wave, returned uniformly (from lane 63 of the scan)
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, dpp_u32<0x111, 0xf>(v, 0xffffffffu));
  v = min(v, dpp_u32<0x112, 0xf>(v, 0xffffffffu));
  v = min(v, dpp_u32<0x114, 0xf>(v, 0xffffffffu));
  v = min(v, dpp_u32<0x118, 0xf>(v, 0xffffffffu));
  v = min(v, dpp_u32<0x142, 0xa>(v, 0xffffffffu));
  v = min(v, dpp_u32<0x143, 0xc>(v, 0xffffffffu));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, dpp_u32<0x111, 0xf>(v, 0u));
  v = max(v, dpp_u32<0x112, 0xf>(v, 0u));
  v = max(v, dpp_u32<0x114, 0xf>(v, 0u));
  v = max(v, dpp_u32<0x118, 0xf>(v, 0u));
  v = max(v, dpp_u32<0x142, 0xa>(v, 0u));
  v = max(v, dpp_u32<0x143, 0xc>(v, 0u));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Block-wide exclusive sums with a single barrier: every wave scans its lanes,
// publishes its total in red[wave]; after the barrier each wave adds the totals
// of the waves before it.  NW = waves per block.  red must not be written again
// before the next barrier every thread passes.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *red, uint32_t *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_sum(v);
  if (lane == 63) red[wid] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = red[w];
    base += (w < wid) ? t : 0u;
    tot += t;
  }
  *total = tot;
  return base + incl - v;
}

// the same for two sums at once (T = long long or double; red holds 2 NW values).
// For double the exclusive value is formed as (prefix of earlier waves) + (inclusive
// - own): rounded, but in a fixed order, so every run gives the same bits.
template <int NW, typename T>
__device__ __forceinline__ void block_excl_sum2(T &a, T &b, T *red, T *ta, T *tb) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const T ia = wave_incl_sum(a), ib = wave_incl_sum(b);
  if (lane == 63) {
    red[wid] = ia;
    red[NW + wid] = ib;
  }
  __syncthreads();
  T ba = 0, bb = 0, sa = 0, sb = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const T va = red[w], vb = red[NW + w];
    if (w < wid) {
      ba += va;
      bb += vb;
    }
    sa += va;
    sb += vb;
  }
  *ta = sa;
  *tb = sb;
  a = ba + (ia - a);
  b = bb + (ib - b);
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024, a
// multiple of 64).  smem needs blockDim.x / 64 entries.  Returns the exclusive
// prefix; *total receives the block sum.  Deterministic order.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *smem, T *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    T o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) smem[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    T s = lane < nw ? smem[lane] : T(0);
    T si = s;
    for (int off = 1; off < 64; off <<= 1) {
      T o = __shfl_up(si, off, 64);
      if (lane >= off) si += o;
    }
    if (lane < nw) smem[lane] = si - s;
    if (lane == nw - 1) smem[63] = si;
  }
  __syncthreads();
  T res = smem[wid] + incl - v;
  T tot = smem[63];
  __syncthreads();
  *total = tot;
  return res;
}

}  // namespace ksum
