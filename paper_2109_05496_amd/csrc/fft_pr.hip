// Phase-retrieval kernels (Section V): a Stockham FFT for the angular-spectrum
// propagator of Eq. (23) and the elementwise pieces of the amplitude
// data-fidelity gradient of Eq. (27) and of FISTA (Algorithm 1).
//
// FFT: lines of length N (a power of two <= 4096) held in LDS, radix-4
// Stockham passes (plus one radix-2 pass when log2 N is odd), each pass reading
// all of its butterfly inputs before a barrier and writing them after, so one
// LDS buffer suffices. A 2-D transform is a row pass (rows are contiguous) and
// a column pass (a tile of C columns loaded transposed into padded LDS). The
// column pass can finish with one of the phase-retrieval steps, and the row
// pass can start with the multiplication by the transfer function, so the
// intermediate arrays make no extra trips through HBM.
// Twiddles and the transfer functions are built on the device in float64
// (the propagation phase 2 pi d / lambda reaches ~3e4 rad) and stored as float2.
#include <hip/hip_runtime.h>

#include "ctv_device.hpp"
#include "ctv_pr.hpp"

namespace ctv {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// DIR = -1: forward (exp(-2 pi i ...)); DIR = +1: inverse (unnormalised).
template <int DIR>
__device__ __forceinline__ float2 twiddle(const float2* tw, int idx) {
  const float2 w = tw[idx];
  return DIR < 0 ? w : conjf2(w);
}

// y_k = sum_r a_r exp(DIR 2 pi i r k / 4)
template <int DIR>
__device__ __forceinline__ void radix4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
  const float2 d = csub(a1, a3);
  // forward: multiply by -i; inverse: by +i
  const float2 t3 = DIR < 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

constexpr int kThreads = 256;
constexpr int kMaxB4 = 8;   // radix-4 butterflies per thread per pass (lines * N <= 8192)
constexpr int kMaxB2 = 16;  // radix-2 butterflies per thread per pass

// Transform `lines` lines of length N stored at s[l*LS + e].
template <int DIR>
__device__ void lds_fft(float2* s, int N, int lines, int LS, const float2* __restrict__ tw) {
  const int tid = threadIdx.x;
  int Ns = 1;
  const int q4 = N >> 2;
  const int total4 = lines * q4;
  while (Ns * 4 <= N) {
    float2 v[kMaxB4][4];
    int dst[kMaxB4];
#pragma unroll
    for (int c = 0; c < kMaxB4; ++c) {
      const int t = tid + c * kThreads;
      dst[c] = -1;
      if (t < total4) {
        const int l = t / q4, j = t - l * q4;
        const float2* L = s + l * LS;
        const int k = j & (Ns - 1);
        const int step = (N / (4 * Ns)) * k;
        float2 a0 = L[j], a1 = L[j + q4], a2 = L[j + 2 * q4], a3 = L[j + 3 * q4];
        if (k) {
          a1 = cmul(a1, twiddle<DIR>(tw, step));
          a2 = cmul(a2, twiddle<DIR>(tw, 2 * step));
          a3 = cmul(a3, twiddle<DIR>(tw, 3 * step));
        }
        radix4<DIR>(a0, a1, a2, a3);
        v[c][0] = a0;
        v[c][1] = a1;
        v[c][2] = a2;
        v[c][3] = a3;
        dst[c] = l * LS + ((j - k) << 2) + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxB4; ++c) {
      if (dst[c] >= 0) {
        s[dst[c]] = v[c][0];
        s[dst[c] + Ns] = v[c][1];
        s[dst[c] + 2 * Ns] = v[c][2];
        s[dst[c] + 3 * Ns] = v[c][3];
      }
    }
    __syncthreads();
    Ns *= 4;
  }
  if (Ns < N) {  // one radix-2 pass (log2 N odd)
    const int q2 = N >> 1;
    const int total2 = lines * q2;
    float2 v0[kMaxB2], v1[kMaxB2];
    int dst[kMaxB2];
#pragma unroll
    for (int c = 0; c < kMaxB2; ++c) {
      const int t = tid + c * kThreads;
      dst[c] = -1;
      if (t < total2) {
        const int l = t / q2, j = t - l * q2;
        const float2* L = s + l * LS;
        const int k = j & (Ns - 1);
        float2 a0 = L[j], a1 = L[j + q2];
        if (k) a1 = cmul(a1, twiddle<DIR>(tw, (N / (2 * Ns)) * k));
        v0[c] = cadd(a0, a1);
        v1[c] = csub(a0, a1);
        dst[c] = l * LS + ((j - k) << 1) + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxB2; ++c) {
      if (dst[c] >= 0) {
        s[dst[c]] = v0[c];
        s[dst[c] + Ns] = v1[c];
      }
    }
    __syncthreads();
  }
}

template <int DIR, int PRE>
__global__ __launch_bounds__(kThreads) void fft_rows_kernel(FftArgs a) {
  extern __shared__ float2 s[];
  const int N = a.n, LS = N + 1;
  const int img = blockIdx.y;
  const int row0 = blockIdx.x * a.lines;
  const float2* in = a.in + (long long)img * a.img_stride;
  float2* out = a.out + (long long)img * a.img_stride;
  const float2* H = a.H ? a.H + (long long)img * a.H_stride : nullptr;
  for (int t = threadIdx.x; t < a.lines * N; t += kThreads) {
    const int l = t / N, c = t - l * N;
    const long long p = (long long)(row0 + l) * N + c;
    float2 v = in[p];
    if (PRE == kPreMulH) v = cmul(v, H[p]);
    s[l * LS + c] = v;
  }
  __syncthreads();
  lds_fft<DIR>(s, N, a.lines, LS, a.tw);
  for (int t = threadIdx.x; t < a.lines * N; t += kThreads) {
    const int l = t / N, c = t - l * N;
    out[(long long)(row0 + l) * N + c] = s[l * LS + c];
  }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
  return t;
}

template <int DIR, int POST>
__global__ __launch_bounds__(kThreads) void fft_cols_kernel(FftArgs a) {
  extern __shared__ float2 s[];
  __shared__ double red[kThreads / 64];
  const int M = a.m, N = a.n, C = a.lines, LS = M + 1;
  const int img = blockIdx.y;
  const int c0 = xcd_remap(blockIdx.x, gridDim.x) * C;
  const long long base = (long long)img * a.img_stride;
  const float2* in = a.in + base;
  for (int t = threadIdx.x; t < M * C; t += kThreads) {
    const int i = t / C, cc = t - i * C;
    s[cc * LS + i] = in[(long long)i * N + c0 + cc];
  }
  __syncthreads();
  lds_fft<DIR>(s, M, C, LS, a.tw);
  double loss = 0.0;
  for (int t = threadIdx.x; t < M * C; t += kThreads) {
    const int i = t / C, cc = t - i * C;
    const long long p = (long long)i * N + c0 + cc;
    float2 v = s[cc * LS + i];
    v.x *= a.scale;
    v.y *= a.scale;
    if (POST == kPostStore) {
      a.out[base + p] = v;
    } else if (POST == kPostResidual) {
      // (A x / |A x|) (|A x| - sqrt(y)), the bracket of Eq. (27); unit phasor at 0
      const float am = sqrtf(v.x * v.x + v.y * v.y);
      const float sy = a.sy[(long long)img * a.sy_stride + p];
      const float r = am - sy;
      float2 ph = make_float2(1.0f, 0.0f);
      if (am > 0.0f) ph = make_float2(v.x / am, v.y / am);
      a.out[base + p] = make_float2(ph.x * r, ph.y * r);
      loss += 0.5 * (double)r * (double)r;
    } else if (POST == kPostAccumulate) {
      const float2 w = cmul(conjf2(a.H[(long long)img * a.H_stride + p]), v);
      if (a.accumulate) {
        const float2 o = a.acc[p];
        a.acc[p] = cadd(o, w);
      } else {
        a.acc[p] = w;
      }
    } else {  // kPostStep: out = z - gamma * v
      const float2 z = a.z[p];
      a.out[base + p] = make_float2(fmaf(-a.gamma, v.x, z.x), fmaf(-a.gamma, v.y, z.y));
    }
  }
  if (POST == kPostResidual) {
    const double tot = block_sum(loss, red);
    if (threadIdx.x == 0) a.partial[(long long)img * gridDim.x + blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(256) void twiddle_kernel(float2* tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double sn, cs;
  sincospi(-2.0 * (double)k / (double)N, &sn, &cs);
  tw[k] = make_float2((float)cs, (float)sn);
}

// H_d(f_x, f_y) of Eq. (23) on the unshifted FFT frequency grid; zero on the
// evanescent band. Frequencies as numpy.fft.fftfreq(n, pixel).
__global__ __launch_bounds__(256) void transfer_kernel(float2* H, int m, int n, double dist, double wavelength,
                                                       double pixel) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)m * n) return;
  const int i = (int)(p / n), j = (int)(p - (long long)i * n);
  const double fy = (double)(i < (m + 1) / 2 ? i : i - m) / ((double)m * pixel);
  const double fx = (double)(j < (n + 1) / 2 ? j : j - n) / ((double)n * pixel);
  const double arg = 1.0 - (wavelength * fx) * (wavelength * fx) - (wavelength * fy) * (wavelength * fy);
  float2 h = make_float2(0.0f, 0.0f);
  if (arg > 0.0) {
    const double ph = 2.0 * dist / wavelength * sqrt(arg);  // phase / pi
    double sn, cs;
    sincospi(ph, &sn, &cs);
    h = make_float2((float)cs, (float)sn);
  }
  H[p] = h;
}

__global__ __launch_bounds__(256) void sqrt_y_kernel(const float* __restrict__ y, float* __restrict__ sy,
                                                     float2* __restrict__ syc, long long total) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const float v = sqrtf(fmaxf(y[p], 0.0f));
  sy[p] = v;
  if (syc) syc[p] = make_float2(v, 0.0f);
}

// z = x + beta (x - x_prev) (Algorithm 1, line 5); also copies x to x_prev.
__global__ __launch_bounds__(256) void fista_kernel(const float2* __restrict__ x, float2* __restrict__ xprev,
                                                    float2* __restrict__ z, float beta, long long total) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const float2 xv = x[p], xp = xprev[p];
  z[p] = make_float2(fmaf(beta, xv.x - xp.x, xv.x), fmaf(beta, xv.y - xp.y, xv.y));
  xprev[p] = xv;
}

__global__ void loss_final_kernel(const double* __restrict__ partial, int count, float* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < count; ++i) s += partial[i];
  *out = (float)s;
}

__global__ __launch_bounds__(256) void copy_c_kernel(const float2* __restrict__ a, float2* __restrict__ b,
                                                     long long total) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < total) b[p] = a[p];
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

bool fft_size_ok(int v) { return v >= 2 && v <= 4096 && (v & (v - 1)) == 0; }

int fft_row_lines(int m, int n, int batch) {
  int lines = std::max(1, 8192 / n);
  while (lines > 1 && (lines > m || (long long)(m / lines) * batch < 512)) lines >>= 1;
  return lines;
}

int fft_col_lines(int m, int n) {
  int c = std::max(1, std::min(8, 8192 / m));
  while (c > n) c >>= 1;
  return c;
}

hipError_t launch_fft_rows(FftArgs a, int dir, int pre, int batch, hipStream_t s) {
  a.lines = fft_row_lines(a.m, a.n, batch);
  const dim3 grid((unsigned)(a.m / a.lines), (unsigned)batch);
  const size_t lds = (size_t)a.lines * (a.n + 1) * sizeof(float2);
  if (dir < 0) {
    if (pre == kPreMulH) hipLaunchKernelGGL((fft_rows_kernel<-1, kPreMulH>), grid, dim3(kThreads), lds, s, a);
    else hipLaunchKernelGGL((fft_rows_kernel<-1, kPreNone>), grid, dim3(kThreads), lds, s, a);
  } else {
    if (pre == kPreMulH) hipLaunchKernelGGL((fft_rows_kernel<1, kPreMulH>), grid, dim3(kThreads), lds, s, a);
    else hipLaunchKernelGGL((fft_rows_kernel<1, kPreNone>), grid, dim3(kThreads), lds, s, a);
  }
  return hipGetLastError();
}

int fft_col_blocks(int m, int n) { return n / fft_col_lines(m, n); }

hipError_t launch_fft_cols(FftArgs a, int dir, int post, int batch, hipStream_t s) {
  a.lines = fft_col_lines(a.m, a.n);
  const dim3 grid((unsigned)(a.n / a.lines), (unsigned)batch);
  const size_t lds = (size_t)a.lines * (a.m + 1) * sizeof(float2);
#define CTV_COLS(D_)                                                                                     \
  switch (post) {                                                                                        \
    case kPostStore: hipLaunchKernelGGL((fft_cols_kernel<D_, kPostStore>), grid, dim3(kThreads), lds, s, a); break; \
    case kPostResidual: hipLaunchKernelGGL((fft_cols_kernel<D_, kPostResidual>), grid, dim3(kThreads), lds, s, a); break; \
    case kPostAccumulate: hipLaunchKernelGGL((fft_cols_kernel<D_, kPostAccumulate>), grid, dim3(kThreads), lds, s, a); break; \
    default: hipLaunchKernelGGL((fft_cols_kernel<D_, kPostStep>), grid, dim3(kThreads), lds, s, a); break; \
  }
  if (dir < 0) {
    CTV_COLS(-1)
  } else {
    CTV_COLS(1)
  }
#undef CTV_COLS
  return hipGetLastError();
}

hipError_t launch_twiddles(float2* tw, int N, hipStream_t s) {
  hipLaunchKernelGGL(twiddle_kernel, dim3((N + 255) / 256), dim3(256), 0, s, tw, N);
  return hipGetLastError();
}

hipError_t launch_transfer(float2* H, int m, int n, double dist, double wavelength, double pixel, hipStream_t s) {
  const long long total = (long long)m * n;
  hipLaunchKernelGGL(transfer_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, H, m, n, dist,
                     wavelength, pixel);
  return hipGetLastError();
}

hipError_t launch_sqrt_y(const float* y, float* sy, float2* syc, long long total, hipStream_t s) {
  hipLaunchKernelGGL(sqrt_y_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, y, sy, syc, total);
  return hipGetLastError();
}

hipError_t launch_fista(const float2* x, float2* xprev, float2* z, float beta, long long total, hipStream_t s) {
  hipLaunchKernelGGL(fista_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, xprev, z, beta, total);
  return hipGetLastError();
}

hipError_t launch_loss_final(const double* partial, int count, float* out, hipStream_t s) {
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, partial, count, out);
  return hipGetLastError();
}

hipError_t launch_copy_c(const float2* a, float2* b, long long total, hipStream_t s) {
  hipLaunchKernelGGL(copy_c_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, b, total);
  return hipGetLastError();
}

int fft_log2(int v) { return ilog2(v); }

}  // namespace ctv
