// Argument block and launchers of the reverse-mode kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctv_kernels.hpp"
#include "ctv_types.hpp"

namespace ctv {

struct AdjStepArgs {
  const float* b;         // chunk base, complex64
  const uint8_t* mask;    // [m][n] or nullptr
  const float* r;         // dual state whose plane 1 is r_k (reverse step; nullptr = zero)
                          // or whose plane 0 is q_K (output step)
  const float* adj_in;    // adjoint state [2][m][n][4]: (A, B)
  float* adj_out;         // same layout, nullptr on the last reverse step
  float* grad_b;          // complex64, read-modify-write
  const float* grad_x;    // complex64 incoming gradient (output step)
  double* lam_acc;        // [chunk][tiles_per_img]
  int m, n, tiles_x, tiles_per_img;
  float beta;             // beta_{k-1}
  Radii R;
  float lam[kPlainChunk];
  float c[kPlainChunk];   // 1/(8 lambda)
  float cc[kPlainChunk];  // 1/(8 lambda^2) (0 for lambda = 0)
};

int adj_tile_rows();
int adj_halo();
hipError_t launch_adj_step(const AdjStepArgs& a, int kind, int constr, int batch, hipStream_t s);
hipError_t launch_adj_output(const AdjStepArgs& a, int constr, int batch, hipStream_t s);
hipError_t launch_pc_vjp(const float* b, const uint8_t* mask, const float* xbar, float* gb, long long px, int batch,
                         int constr, hipStream_t s);
hipError_t launch_lam_final(const double* acc, int tiles_per_img, int batch, float* out, hipStream_t s);
hipError_t launch_zero_f32(float* p, long long count, hipStream_t s);

}  // namespace ctv
