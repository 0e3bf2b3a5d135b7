// Argument block and launchers of the FFT / phase-retrieval kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace ctv {

// kPreExtrapolate: the input is x + beta (x - in2) (Algorithm 1's z update),
// also stored to zout at the same positions.
enum FftPre { kPreNone = 0, kPreMulH = 1, kPreMulConjH = 2, kPreExtrapolate = 3 };
// kPostAccumulateAll: acc (+)= sum over n_acc images of conj(H_img) * transform
// (the images are looped inside one launch, so there is no race on acc).
// kPostReplace: sqrt(y) times the unit phasor of the value (the measured-modulus
// projection in the sensor plane); kPostProjC: P_C of Eq. (26) (constr).
enum FftPost { kPostStore = 0, kPostResidual = 1, kPostAccumulateAll = 2, kPostStep = 3, kPostReplace = 4,
               kPostProjC = 5 };

// One line pass: `lines` lines of length N along the contiguous axis of each
// batch image. Element p of input image img is in[img * in_stride + p], of
// output image img out[img * img_stride + p].
struct FftArgs {
  const float2* in;
  float2* out;
  long long in_stride;    // elements between batch images of in (0 = one input shared by all)
  long long img_stride;   // elements between batch images of out
  long long lines;        // set by the launcher
  const float2* tw;       // exp(-2 pi i k / N), k < N
  int pre, post;          // FftPre / FftPost
  const float2* H;        // PRE multiply / POST accumulate table (same layout as the pass)
  long long H_stride;     // per-image stride of H (0 = shared)
  const float* sy;        // sqrt(y) for the residual (same layout as the pass output)
  long long sy_stride;
  float2* acc;            // accumulation target
  const float2* z;        // base point of the gradient step
  float gamma;
  float scale;            // applied to the pass output
  double* partial;        // residual loss partials, one per block (and image)
  int accumulate;         // 0: acc = w, 1: acc += w
  int n_acc;              // images summed by kPostAccumulateAll
  int constr;             // kPostProjC: 0 = C^{m x n} (store), 1 = |x| <= 1
  const float2* in2;      // kPreExtrapolate: the previous iterate (layout and stride of in)
  float2* zout;           // kPreExtrapolate: where the extrapolated input is stored
  float beta;             // kPreExtrapolate: the momentum weight
};

bool fft_size_ok(int v);
int fft_line_blocks(int N, long long lines);
hipError_t launch_fft_lines(FftArgs a, int N, long long lines, int dir, int batch, hipStream_t s);
hipError_t launch_transpose(const float2* in, float2* out, int R, int C, int batch, hipStream_t s);
// Second pass of a 2-D transform: input images [N][W] (a.in, stride a.in_stride),
// FFT along the N-long columns, output transposed [W][N] (a.out / epilogue in
// that layout): one column-pass launch; for N <= 16 and for the accumulate-all
// epilogue a transpose into tmp (N * W elements per image) and a line pass.
hipError_t launch_fft_second(FftArgs a, int N, long long W, int dir, int batch, float2* tmp, hipStream_t s);
int fft_second_blocks(int N, long long W);
// Inverse DFT of every N-long column of [N][W] images (N >= 32), the Eq. (27)
// residual (a.sy, a.sy_stride, a.scale, loss partials in a.partial with
// fft_second_blocks(N, W) blocks per image), forward DFT back; out keeps the
// [N][W] layout.
hipError_t launch_fft_roundtrip(FftArgs a, int N, long long W, int batch, hipStream_t s);
// Along the N-long lines (N >= 32) of the a.n_acc images a.in (stride
// a.in_stride): out = IDFT(sum_img conj(H_img) (.) a.scale * DFT(line of img)),
// unscaled, one [lines][N] image (H, H_stride as for kPostAccumulateAll).
hipError_t launch_fft_acc_inverse(FftArgs a, int N, long long lines, hipStream_t s);
hipError_t launch_twiddles(float2* tw, int N, hipStream_t s);
hipError_t launch_transfer_t(float2* Ht, int m, int n, double dist, double wavelength, double pixel, hipStream_t s);
hipError_t launch_sqrt_y(const float* y, float* sy, float2* syc, long long total, hipStream_t s);
hipError_t launch_loss_final(const double* partial, int count, float* out, hipStream_t s);
hipError_t launch_copy_c(const float2* a, float2* b, long long total, hipStream_t s);
// Line search helpers: out[j] = sum_i partial[i * stride + j] (j < width <= 64, float64,
// fixed order); v = z - gamma g; kLsBlocks partial pairs (Re<g, x - z>, ||x - z||^2).
constexpr int kLsBlocks = 512;
hipError_t launch_fill_f32(float* p, float v, long long count, hipStream_t s);
hipError_t launch_sum_d(const double* partial, int count, int stride, int width, double* out, hipStream_t s);
hipError_t launch_grad_step(const float2* z, const float2* g, float gamma, float2* v, long long total, hipStream_t s);
hipError_t launch_ls_dots(const float2* g, const float2* x, const float2* z, long long total, double* partial,
                          hipStream_t s);

}  // namespace ctv
