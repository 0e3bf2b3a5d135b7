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
void momentum_table(int kmax, std::vector<float>& beta);
float step_of(float lam);
ctv_status choose_tiling(const ctv_params* p, int m, int n, int batch, Tiling* out);
size_t state_bytes(long long batch, long long m, long long n);
int gap_blocks_per_image(long long px);
size_t denoise_ws_bytes(int batch, int m, int n);

}  // namespace ctv
