// Tile job description and wave-level helpers shared by the forward tile
// kernels (column-register tiles and the row-sweep tile).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctv_types.hpp"

namespace ctv {

constexpr int kRW = 64;  // columns of a tile region: one per lane of a wave64

struct TileJob {
  const float2* b;       // image (m x n)
  const uint8_t* mask;   // image support or nullptr
  const float4* st_in;   // [2][m][n] (q plane, r plane) or nullptr = cold start
  float4* st_out;        // [2][m][n] or nullptr
  float2* x;             // Eq. (18) output or nullptr
  int m, n;
  int tx, ty;
  float lam, c;
  Radii R;
  int T;
  float4* r_hist;          // r after each fused iteration (plane 1 of consecutive states), or nullptr
  long long hist_stride;   // float4 elements from one iteration's state to the next
};

// Whole-wave lane shifts through DPP (row_shr / row_shl across the wave with
// bound control): the neighbouring column's value, 0 past the wave's edge.
__device__ __forceinline__ float lane_from_left(float v) {   // lane i <- lane i-1 (lane 0 <- 0)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {  // lane i <- lane i+1 (lane 63 <- 0)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Bits [max(a, 0), min(b, n)) set: the rows i of a wave with a <= i < b.
__device__ __forceinline__ unsigned row_bits(int a, int b, int n) {
  a = min(max(a, 0), n);
  b = min(max(b, 0), n);
  return ((1u << b) - 1u) & ~((1u << a) - 1u);
}

}  // namespace ctv
