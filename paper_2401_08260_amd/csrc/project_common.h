// Shared pieces of the projection GEMMs (FP32 and split-BF16): the loader of the
// point tile and the control block of the persistent tile queue.
#pragma once

#include "device_common.h"
#include "internal.h"

namespace ksum {

// Loads 4 consecutive columns of one row of a point tile: element e of a tile of
// rows [l0, ...) and columns [k0, k0 + 16) is row l0 + e / 4, columns k0 + 4 (e % 4) ..+3
// (zero outside the union or beyond d), VW elements per load (VW = 4: 16-byte
// loads, d % 4 == 0; VW = 2: 8-byte loads, d even; VW = 1: any d).
template <typename InT, int VW>
struct PointLoader {
  const InT *x, *y;
  int64_t N, M, L;
  int d;

  __device__ __forceinline__ float4 load1(int64_t l0, int k0, int e) const {
    const int row = e >> 2, k4 = (e & 3) * 4;
    const int64_t l = l0 + row;
    const int k = k0 + k4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l < L) {
      const InT *src = (l < M) ? (y + l * (int64_t)d) : (x + (l - M) * (int64_t)d);
      if constexpr (VW == 4) {
        if (k < d) v = *reinterpret_cast<const float4 *>(src + k);
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
    }
    return v;
  }
};

// 16-byte store of four projections into Z with the non-temporal hint: Z is far
// larger than the caches and is read back by the next stage only after the whole
// GEMM, so keeping it out of the caches loses nothing
__device__ __forceinline__ void store_z4(float *dst, float4 v) {
  typedef float nt4 __attribute__((ext_vector_type(4)));
  const nt4 nv = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(nv, reinterpret_cast<nt4 *>(dst));
}

struct GemmCtl {
  const float *dirs;
  int d_pad, p0, nsl;
  float *Z;
  int64_t ldz;
  uint32_t *counter;      // tile queue heads, 16 (zeroed before the launch)
  uint32_t *part;         // [gridDim.x][nsl][2] per-block min / max keys
  int n_col_tiles, n_row_tiles;
  const uint16_t *dirs_hi, *dirs_lo;   // split-BF16 directions [P_pad][d_pad] (split path only)
  int z_vec4;             // Z rows are 16-byte aligned (ldz % 4 == 0): 16-byte stores
  const uint16_t *dirs_t;  // step-tiled split directions [d_pad / 16][a_rows][32], or null
  const uint16_t *pts_t;   // step-tiled split points [d_pad / 16][b_rows][32] in union order (zero
                           // past L and d), or null: the points are split inside the GEMM
  int64_t a_rows, b_rows;
};

}  // namespace ksum
