// Argument block and launchers of the reverse-mode kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctv_kernels.hpp"
#include "ctv_types.hpp"

namespace ctv {

constexpr int kMaxRev = 5;  // reverse steps fused per launch

struct AdjStepArgs {
  const float* b;           // chunk base, complex64
  const uint8_t* mask;      // [m][n] or nullptr
  const float* r[kMaxRev];  // reverse step: per fused step, the dual state whose plane 1 is r_k
                            // (nullptr = zero); output step: r[0] is the state whose plane 0 is q_K
  const float* adj_in;      // adjoint state [2][m][n][4]: (A, B)
  float* adj_out;           // same layout, nullptr after the last reverse step
  float* grad_b;            // complex64, read-modify-write
  const float* grad_x;      // complex64 incoming gradient (output step)
  double* lam_acc;          // [chunk][tiles_per_img]
  int m, n, tiles_x, tiles_per_img;
  int halo;                 // tile halo, >= steps + 1, the same for every launch of a call
  int steps;                // reverse steps in this launch, 1..kMaxRev
  float beta[kMaxRev];      // beta_{k-1} of each fused step k
  Radii R;
  float lam[kPlainChunk];
  float c[kPlainChunk];     // 1/(8 lambda)
  float cc[kPlainChunk];    // 1/(8 lambda^2) (0 for lambda = 0)
  const int* live;          // reverse steps only: [0] = L, [1 .. L] = the tiles (of one image) to run,
                            // or nullptr for all (the grid stays one workgroup per tile of the chunk)
};

int adj_tile_rows();
hipError_t launch_adj_step(const AdjStepArgs& a, int kind, int constr, int batch, hipStream_t s);
hipError_t launch_adj_output(const AdjStepArgs& a, int constr, int batch, hipStream_t s);
hipError_t launch_pc_vjp(const float* b, const uint8_t* mask, const float* xbar, float* gb, long long px, int batch,
                         int constr, hipStream_t s);
hipError_t launch_lam_final(const double* acc, int tiles_per_img, int batch, float* out, hipStream_t s);
hipError_t launch_zero_f32(float* p, long long count, hipStream_t s);

}  // namespace ctv
