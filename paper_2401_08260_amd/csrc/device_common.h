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
