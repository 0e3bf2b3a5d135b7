// Argument block and launchers of the FFT / phase-retrieval kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

namespace ctv {

enum FftPre { kPreNone = 0, kPreMulH = 1 };
enum FftPost { kPostStore = 0, kPostResidual = 1, kPostAccumulate = 2, kPostStep = 3 };

struct FftArgs {
  const float2* in;
  float2* out;
  int m, n;               // array shape; rows pass transforms length n, column pass length m
  long long img_stride;   // elements between batch images of in/out
  const float2* tw;       // twiddles exp(-2 pi i k / N), k < N, for this pass's length
  const float2* H;        // transfer function [m][n] (PRE mul / POST accumulate)
  long long H_stride;     // per-batch-image stride of H (0 = shared)
  const float* sy;        // sqrt(y) for the residual
  long long sy_stride;
  float2* acc;            // accumulation target
  const float2* z;        // base point of the gradient step
  float gamma;
  float scale;            // applied to the column-pass output
  double* partial;        // residual loss partials, one per column block
  int lines;              // set by the launcher
  int accumulate;         // 0: acc = w, 1: acc += w
};

bool fft_size_ok(int v);
int fft_log2(int v);
int fft_col_blocks(int m, int n);
hipError_t launch_fft_rows(FftArgs a, int dir, int pre, int batch, hipStream_t s);
hipError_t launch_fft_cols(FftArgs a, int dir, int post, int batch, hipStream_t s);
hipError_t launch_twiddles(float2* tw, int N, hipStream_t s);
hipError_t launch_transfer(float2* H, int m, int n, double dist, double wavelength, double pixel, hipStream_t s);
hipError_t launch_sqrt_y(const float* y, float* sy, float2* syc, long long total, hipStream_t s);
hipError_t launch_fista(const float2* x, float2* xprev, float2* z, float beta, long long total, hipStream_t s);
hipError_t launch_loss_final(const double* partial, int count, float* out, hipStream_t s);
hipError_t launch_copy_c(const float2* a, float2* b, long long total, hipStream_t s);

}  // namespace ctv
