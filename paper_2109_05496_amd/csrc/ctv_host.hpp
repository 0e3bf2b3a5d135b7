// Host-side helpers shared by the C ABI translation units (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ctv.h"
#include "ctv_kernels.hpp"
#include "ctv_types.hpp"

namespace ctv {

struct Tiling {
  int T;            // iterations fused per launch
  TileShape shape;  // tile kernel variant and region rows (64 columns)
};

ctv_status fail(ctv_status st, const std::string& msg);
ctv_status hip_fail(hipError_t e, const char* where);
ctv_status validate_params(const ctv_params* p);
ctv_status validate_lambda(float lam);
Radii make_radii(int kind, float alpha);
void momentum_table(int method, int kmax, std::vector<float>& beta);
float step_of(float lam);
// Launch configuration for a plain call: the explicit fuse / tile of p, else
// (use_tuned) an entry recorded by ctv_autotune for this problem, else the default.
ctv_status choose_tiling(const ctv_params* p, int m, int n, int batch, Tiling* out, bool use_tuned = false);
// Limits the fusion depth to what the tile shape's halo and the run allow.
void clamp_fuse(Tiling* t, int iters);
// Tuning table (autotune.cpp): problem keys and lookup for the current device.
uint64_t plain_tune_key(const ctv_params* p, int batch, int m, int n);
uint64_t batched_tune_key(const ctv_image_desc* d, int count, const ctv_params* common);
bool tuned_lookup(uint64_t key, Tiling* out);
// Iterations for the next launch when `left` iterations remain in a run that
// takes at most T per launch: the fewest launches, with the iterations spread
// evenly (8 + 1 becomes 5 + 4; a smaller fusion depth also means a smaller halo).
inline int even_split(int T, int left) {
  if (left <= 0) return 0;
  const int launches = (left + T - 1) / T;
  return (left + launches - 1) / launches;
}
size_t state_bytes(long long batch, long long m, long long n);
int gap_blocks_per_image(long long px);
size_t denoise_ws_bytes(int batch, int m, int n);
// One launch of the plain fused kernel: iterations k+1 .. k+Tl on a chunk of
// cb <= 32 images (per-image lambdas lam[0..cb)), from state src (nullptr =
// cold start) into dst (nullptr = not stored); x != nullptr adds Eq. (18).
// r_hist != nullptr (8 x 8 column tile only) also stores r after each fused
// iteration i into plane 1 of the state at r_hist + i * r_hist_stride floats.
// live (column tiles only): the live-tile list of this tiling; the other tiles
// are not run, so src and dst must already hold their (zero) values.
ctv_status fgp_launch(const ctv_params* p, const Tiling& tl, int cb, int m, int n, const float* b,
                      const uint8_t* support, const float* lam, const std::vector<float>& beta, int k, int Tl,
                      const float* src, float* dst, float* x, hipStream_t s, float* r_hist = nullptr,
                      long long r_hist_stride = 0, const int* live = nullptr);

}  // namespace ctv
