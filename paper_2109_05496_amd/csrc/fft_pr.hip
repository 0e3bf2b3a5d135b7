// Phase-retrieval kernels (Section V): a Stockham FFT for the angular-spectrum
// propagator of Eq. (23) and the elementwise pieces of the amplitude
// data-fidelity gradient of Eq. (27) and of FISTA (Algorithm 1).
//
// FFT of lines of length N = 2^L along rows (the contiguous axis):
//   * N >= 32: N/16 threads per line. Radix-16 Stockham passes run in
//     registers (a 16-point DFT per thread per pass), followed by one radix-8,
//     -4 or -2 pass when L is not a multiple of 4. The first pass reads its
//     inputs straight from global memory and the last pass writes straight to
//     global memory, both coalesced; only the passes in between exchange data
//     through LDS (2 exchanges for N = 1024).
//   * N <= 16: one thread per line, one DFT in registers.
// A 2-D transform is a row pass, a tiled transpose and a second row pass, so
// the spectrum lives transposed ([n][m]); the inverse transform starts from
// that layout and ends in the natural one, and the transfer functions are
// built transposed, so each FFT2 / IFFT2 costs two line passes and one
// transpose. The first pass can multiply by a table on load (H_d), the last can
// store, form the Eq. (27) residual with float64 loss partials, accumulate
// conj(H_d) * (.), or take the gradient step z - gamma * (.).
// Twiddles and transfer functions are built on the device in float64 (the
// propagation phase 2 pi d / lambda_s reaches ~3e4 rad) and stored as float2.
#include <climits>
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

// multiply by exp(DIR * i * pi / 2) = DIR < 0 ? -i : +i
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  const float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

// X_k = sum_r a_r exp(DIR 2 pi i r k / 4)
template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot90<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// exp(DIR 2 pi i t / 16) for t = 0..15 (constants, float64-rounded)
template <int DIR>
__device__ __forceinline__ float2 w16(int t) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
  const float cs[16] = {1.0f, c1, h, s1, 0.0f, -s1, -h, -c1, -1.0f, -c1, -h, -s1, 0.0f, s1, h, c1};
  const float sn[16] = {0.0f, s1, h, c1, 1.0f, c1, h, s1, 0.0f, -s1, -h, -c1, -1.0f, -c1, -h, -s1};
  return make_float2(cs[t & 15], DIR < 0 ? -sn[t & 15] : sn[t & 15]);
}

// In-register DFT of length R in {2, 4, 8, 16}: v[k] <- sum_r v[r] exp(DIR 2 pi i r k / R)
template <int R, int DIR>
__device__ __forceinline__ void dft(float2 (&v)[16]) {
  if (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else if (R == 8) {
    // n = 2 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle W8^(n2 k1), DFT2 over n2
    float2 y[2][4];
#pragma unroll
    for (int n2 = 0; n2 < 2; ++n2) {
      float2 a0 = v[n2], a1 = v[2 + n2], a2 = v[4 + n2], a3 = v[6 + n2];
      dft4<DIR>(a0, a1, a2, a3);
      y[n2][0] = a0;
      y[n2][1] = cmul(a1, w16<DIR>(2 * n2));
      y[n2][2] = cmul(a2, w16<DIR>(4 * n2));
      y[n2][3] = cmul(a3, w16<DIR>(6 * n2));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      v[k1] = cadd(y[0][k1], y[1][k1]);
      v[k1 + 4] = csub(y[0][k1], y[1][k1]);
    }
  } else {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle W16^(n2 k1), DFT4 over n2
    float2 y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
      dft4<DIR>(a0, a1, a2, a3);
      y[n2][0] = a0;
      y[n2][1] = n2 ? cmul(a1, w16<DIR>(n2)) : a1;
      y[n2][2] = n2 ? cmul(a2, w16<DIR>(2 * n2)) : a2;
      y[n2][3] = n2 ? cmul(a3, w16<DIR>(3 * n2)) : a3;
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
      dft4<DIR>(a0, a1, a2, a3);
      v[k1] = a0;
      v[k1 + 4] = a1;
      v[k1 + 8] = a2;
      v[k1 + 12] = a3;
    }
  }
}

constexpr int kThreads = 256;

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

// The last-pass epilogue for CNT elements of image `img` at linear indices
// lbase + pos[r]. The epilogue kind is tested once for the whole block, so the
// side loads (sqrt(y) or z) of all CNT elements are in flight together instead
// of each waiting in a branch of its own.
template <int CNT>
__device__ __forceinline__ void post_block(const FftArgs& a, int img, long long lbase, const int (&pos)[16],
                                           float2 (&v)[16], double& loss) {
#pragma unroll
  for (int r = 0; r < CNT; ++r) v[r] = make_float2(v[r].x * a.scale, v[r].y * a.scale);
  float2* out = a.out + (long long)img * a.img_stride + lbase;
  if (a.post == kPostStore) {
#pragma unroll
    for (int r = 0; r < CNT; ++r) out[pos[r]] = v[r];
  } else if (a.post == kPostResidual || a.post == kPostReplace) {
    // residual: (A x / |A x|)(|A x| - sqrt(y)), the bracket of Eq. (27);
    // replace: (A x / |A x|) sqrt(y), the measured modulus with the phase kept;
    // both with the unit phasor where A x = 0
    const float* sy = a.sy + (long long)img * a.sy_stride + lbase;
    float y[16];
#pragma unroll
    for (int r = 0; r < CNT; ++r) y[r] = sy[pos[r]];
    const bool res = a.post == kPostResidual;
#pragma unroll
    for (int r = 0; r < CNT; ++r) {
      const float am = sqrtf(v[r].x * v[r].x + v[r].y * v[r].y);
      const float mag = res ? am - y[r] : y[r];
      float2 ph = make_float2(1.0f, 0.0f);
      if (am > 0.0f) ph = make_float2(v[r].x / am, v[r].y / am);
      out[pos[r]] = make_float2(ph.x * mag, ph.y * mag);
      if (res) loss += 0.5 * (double)mag * (double)mag;
    }
  } else if (a.post == kPostStep) {
    const float2* z = a.z + lbase;
    float2 zz[16];
#pragma unroll
    for (int r = 0; r < CNT; ++r) zz[r] = z[pos[r]];
#pragma unroll
    for (int r = 0; r < CNT; ++r)
      out[pos[r]] = make_float2(fmaf(-a.gamma, v[r].x, zz[r].x), fmaf(-a.gamma, v[r].y, zz[r].y));
  } else {  // kPostProjC: v / max{1, |v|} (Eq. 26)
#pragma unroll
    for (int r = 0; r < CNT; ++r) {
      float2 w = v[r];
      if (a.constr) {
        const float am = sqrtf(w.x * w.x + w.y * w.y);
        if (am > 1.0f) w = make_float2(w.x / am, w.y / am);
      }
      out[pos[r]] = w;
    }
  }
}

// Loads CNT elements of image `img` at p0 + r * STRIDE into v, multiplied by H
// or conj(H) at the same positions, or extrapolated as x + beta (x - x_prev)
// (and stored), when a.pre asks for it (all loads issued before the first use).
template <int CNT, int STRIDE>
__device__ __forceinline__ void load_pre(const FftArgs& a, int img, long long p0, float2 (&v)[16]) {
  const float2* in = a.in + (long long)img * a.in_stride + p0;
#pragma unroll
  for (int r = 0; r < CNT; ++r) v[r] = in[r * STRIDE];
  if (a.pre == kPreExtrapolate) {
    const float2* xp = a.in2 + (long long)img * a.in_stride + p0;
    float2* zo = a.zout + (long long)img * a.in_stride + p0;
    float2 u[16];
#pragma unroll
    for (int r = 0; r < CNT; ++r) u[r] = xp[r * STRIDE];
#pragma unroll
    for (int r = 0; r < CNT; ++r) {
      v[r] = make_float2(fmaf(a.beta, v[r].x - u[r].x, v[r].x), fmaf(a.beta, v[r].y - u[r].y, v[r].y));
      zo[r * STRIDE] = v[r];
    }
  } else if (a.pre != kPreNone) {
    const float2* H = a.H + (long long)img * a.H_stride + p0;
    float2 h[16];
#pragma unroll
    for (int r = 0; r < CNT; ++r) h[r] = H[r * STRIDE];
    const bool cj = a.pre != kPreMulH;
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = cmul(v[r], cj ? conjf2(h[r]) : h[r]);
  }
}

// One Stockham pass of radix R over an LDS line (Ns = size of the sub-transforms
// already done); the thread handles butterflies j0, j0 + TPL, ... < N/R.
// LDS index with one pad element per 16: the strided writes of a pass spread
// over the banks instead of landing on one.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// exp(-+2 pi i idx / N) (sign by DIR) for 0 <= idx < N from the half table
// twh[k] = exp(-2 pi i k / N), k < N/2, staged in LDS: the second half is the
// first negated.
template <int N, int DIR>
__device__ __forceinline__ float2 tw_half(const float2* twh, int idx) {
  const float2 w = twh[idx & (N / 2 - 1)];
  const unsigned neg = (unsigned)(idx & (N / 2)) << (31 - __builtin_ctz(N / 2));  // sign bit for the second half
  const float x = __uint_as_float(__float_as_uint(w.x) ^ neg);
  const float y = __uint_as_float(__float_as_uint(w.y) ^ neg);
  return DIR < 0 ? make_float2(x, y) : make_float2(x, -y);
}

// The first N/2 twiddles staged into LDS by NT threads: the loads (issued
// before the caller's own) and the LDS stores (after them) are separate, so
// waiting for the twiddles does not hold back the data loads.
template <int N, int NT>
struct TwStage {
  static constexpr int K = (N / 2 + NT - 1) / NT;
  float2 v[K];
  __device__ __forceinline__ void fetch(const float2* __restrict__ tw) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int idx = (int)threadIdx.x + i * NT;
      v[i] = idx < N / 2 ? tw[idx] : make_float2(0.0f, 0.0f);
    }
  }
  __device__ __forceinline__ void store(float2* twh) const {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int idx = (int)threadIdx.x + i * NT;
      if (idx < N / 2) twh[idx] = v[i];
    }
  }
};

template <int N, int R, int DIR, int TPL>
__device__ __forceinline__ void pass_lds(const float2* L, float2 (&v)[16], int j, int Ns, const float2* twh) {
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = L[pidx(j + r * (N / R))];
  const int k = j & (Ns - 1);
  if (k) {
    const int step = (N / (Ns * R)) * k;
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw_half<N, DIR>(twh, r * step));
  }
  dft<R, DIR>(v);
}

// The FFT of one line from the first radix-E pass on (E = 16 or 8 elements per
// thread), the thread's E inputs (line positions lt + r * N/E) already in v,
// twiddles from the LDS half table twh (visible after the first barrier here);
// the E outputs of the last pass are returned in o[] with their positions
// within the line in pos[]. E = 8 gives a line twice the threads (for passes
// over a single image, which otherwise leave each CU a handful of waves).
// OPAQUE_LANE: take the lane index through an empty asm, so that a second
// transform in the same kernel recomputes its LDS and twiddle offsets instead
// of keeping the first one's alive in registers.
template <int N, int DIR, bool OPAQUE_LANE = false, int E = 16>
__device__ __forceinline__ void line_fft_regs(float2* sl, const float2* twh, float2 (&v)[16], float2 (&o)[16],
                                              int (&pos)[16]) {
  static_assert(E == 16 || E == 8, "16 or 8 elements per thread");
  constexpr int TPL = N / E;                   // threads per line
  constexpr int L = (N == 32) ? 5 : (N == 64) ? 6 : (N == 128) ? 7 : (N == 256) ? 8 : (N == 512) ? 9
                  : (N == 1024) ? 10 : (N == 2048) ? 11 : 12;
  constexpr int LE = E == 16 ? 4 : 3;          // log2(E)
  constexpr int PE = L / LE;                   // radix-E passes
  constexpr int RR = 1 << (L % LE);            // remainder radix (1 = none)
  constexpr int NPASS = PE + (RR > 1 ? 1 : 0);  // >= 2 for N >= 32
  int lt = threadIdx.x % TPL;
  if (OPAQUE_LANE) asm volatile("" : "+v"(lt));
  dft<E, DIR>(v);
  int Ns = E;
  __syncthreads();  // the previous use of this LDS line (an earlier image) is finished
#pragma unroll
  for (int r = 0; r < E; ++r) sl[pidx(lt * E + r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int p = 1; p < NPASS; ++p) {
    const bool last = (p == NPASS - 1);
    if (p < PE) {
      pass_lds<N, E, DIR, TPL>(sl, v, lt, Ns, twh);
      const int k = lt & (Ns - 1);
      const int d = (lt - k) * E + k;
      if (!last) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r) sl[pidx(d + r * Ns)] = v[r];
        __syncthreads();
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          o[r] = v[r];
          pos[r] = d + r * Ns;
        }
      }
      Ns *= E;
    } else {
      // remainder pass of radix RR (always the last): E/RR butterflies per thread
      constexpr int B = E / RR;
#pragma unroll
      for (int bb = 0; bb < B; ++bb) {
        float2 w[16];
        const int j = lt + bb * TPL;
        pass_lds<N, RR, DIR, TPL>(sl, w, j, Ns, twh);
        const int k = j & (Ns - 1);
        const int d = (j - k) * RR + k;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          o[bb * RR + r] = w[r];
          pos[bb * RR + r] = d + r * Ns;
        }
      }
      Ns *= RR;
    }
  }
}

// The 16 inputs of this thread's first pass for line `line` of image `img`
// (positions lt + r * N/16), with the pre-operation of a.pre; zeros if !live.
template <int N, int E = 16>
__device__ __forceinline__ void line_load(const FftArgs& a, int img, long long line, bool live, float2 (&v)[16]) {
  constexpr int TPL = N / E;
  const int lt = threadIdx.x % TPL;
  if (live) {
    load_pre<E, TPL>(a, img, line * N + lt, v);
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = make_float2(0.0f, 0.0f);
  }
}

// The same inputs from a line staged in LDS (natural order, pidx positions).
template <int N, int E = 16>
__device__ __forceinline__ void line_from_lds(const float2* sl, float2 (&v)[16]) {
  constexpr int TPL = N / E;
  const int lt = threadIdx.x % TPL;
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = sl[pidx(lt + r * TPL)];
}

template <int N, int DIR, bool ACCALL, int E = 16>
__global__ __launch_bounds__(kThreads) void fft_line_kernel(FftArgs a) {
  constexpr int TPL = N / E;
  constexpr int LPB = kThreads / TPL;          // lines per block
  constexpr int LS = N + N / 16;               // padded LDS line length
  __shared__ float2 s[LPB * LS];
  __shared__ float2 twh[N / 2];
  __shared__ double red[kThreads / 64];
  const int li = threadIdx.x / TPL;
  const long long line = (long long)blockIdx.x * LPB + li;
  const bool live = line < a.lines;
  float2* sl = s + li * LS;
  float2 o[16], v[16];
  int pos[16];
  TwStage<N, kThreads> tws;
  tws.fetch(a.tw);
  if (ACCALL) {
    static_assert(!ACCALL || E == 16, "the accumulate-all pass runs 16 elements per thread");
    // acc (+)= sum over the n_acc images of conj(H_img) * FFT(line of image img)
    float2 sum[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) sum[r] = make_float2(0.0f, 0.0f);
    for (int img = 0; img < a.n_acc; ++img) {
      line_load<N>(a, img, line, live, v);
      if (img == 0) tws.store(twh);
      line_fft_regs<N, DIR>(sl, twh, v, o, pos);
      if (live) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float2 h = a.H[(long long)img * a.H_stride + line * N + pos[r]];
          sum[r] = cadd(sum[r], cmul(conjf2(h), make_float2(o[r].x * a.scale, o[r].y * a.scale)));
        }
      }
    }
    if (live) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long p = line * N + pos[r];
        a.acc[p] = a.accumulate ? cadd(a.acc[p], sum[r]) : sum[r];
      }
    }
    return;
  }
  const int img = blockIdx.y;
  line_load<N, E>(a, img, line, live, v);
  tws.store(twh);
  line_fft_regs<N, DIR, false, E>(sl, twh, v, o, pos);
  double loss = 0.0;
  if (live) post_block<E>(a, img, line * N, pos, o, loss);
  if (a.post == kPostResidual) {
    const double tot = block_sum(loss, red);
    if (threadIdx.x == 0) a.partial[(long long)img * gridDim.x + blockIdx.x] = tot;
  }
}

// Along the lines of [lines][N] images (the m-direction of the transposed
// spectrum layout, N >= 32): the forward DFT of a line of each of the n_acc
// images, scaled by a.scale and multiplied by conj(H_img) at the same
// frequencies, summed over the images (the sum over distances of Eq. (27)),
// then the inverse DFT of that sum along the same line, stored unscaled in
// a.out ([lines][N]) - the accumulate pass and the first inverse pass of the
// gradient in one. G groups of a block transform different images of the same
// line side by side (group g takes images g, g + G, ...), so a line's images
// are in flight together; the group partials are then added in group order
// (for n_acc <= G that is the sequential order over the images) and every
// group runs the inverse (all take part in its barriers), group 0 storing it.
template <int N>
constexpr int acc_groups() { return (kThreads / (N / 16)) < 4 ? (kThreads / (N / 16)) : 4; }
template <int N>
constexpr int acc_lines_per_block() { return (kThreads / (N / 16)) / acc_groups<N>(); }

// ONE: n_acc <= G, every group transforms at most one image (no running sum).
template <int N, bool ONE>
__global__ __launch_bounds__(kThreads) void fft_acc_inverse_kernel(FftArgs a) {
  constexpr int TPL = N / 16;
  constexpr int SLOTS = kThreads / TPL;        // line slots per block
  constexpr int G = acc_groups<N>();           // image groups per line
  constexpr int LPB = acc_lines_per_block<N>();
  constexpr int LS = N + N / 16;
  __shared__ float2 s[SLOTS * LS];
  __shared__ float2 twh[N / 2];
  const int slot = threadIdx.x / TPL;
  const int g = slot % G, li = slot / G;
  const int lt = threadIdx.x % TPL;
  const long long line = (long long)blockIdx.x * LPB + li;
  const bool live = line < a.lines;
  float2* sl = s + slot * LS;
  float2 sum[16], o[16], v[16];
  int pos[16];
  TwStage<N, kThreads> tws;
  tws.fetch(a.tw);
  const int rounds = ONE ? 1 : (a.n_acc + G - 1) / G;  // the same for every group: barriers match
  for (int it = 0; it < rounds; ++it) {
    const int img = g + it * G;
    const bool act = live && img < a.n_acc;
    line_load<N>(a, act ? img : 0, line, act, v);
    if (it == 0) tws.store(twh);
    line_fft_regs<N, -1>(sl, twh, v, o, pos);
    float2 h[16];
    const float2* H = a.H + (long long)(act ? img : 0) * a.H_stride + line * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) h[r] = act ? H[pos[r]] : make_float2(0.0f, 0.0f);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 t = cmul(conjf2(h[r]), make_float2(o[r].x * a.scale, o[r].y * a.scale));
      sum[r] = it == 0 ? t : cadd(sum[r], t);
    }
  }
  __syncthreads();  // every group's last pass has read its line
#pragma unroll
  for (int r = 0; r < 16; ++r) sl[pidx(pos[r])] = sum[r];
  __syncthreads();
  const float2* s0 = s + (li * G) * LS;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int p = pidx(lt + r * TPL);
    float2 t = s0[p];
#pragma unroll
    for (int gg = 1; gg < G; ++gg) t = cadd(t, s0[gg * LS + p]);
    v[r] = t;
  }
  line_fft_regs<N, 1, true>(sl, twh, v, o, pos);
  if (live && g == 0) {
    float2* out = a.out + line * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) out[pos[r]] = o[r];
  }
}

// N <= 16: one thread per line.
template <int N, int DIR, bool ACCALL>
__global__ __launch_bounds__(kThreads) void fft_small_kernel(FftArgs a) {
  __shared__ double red[kThreads / 64];
  const long long line = (long long)blockIdx.x * kThreads + threadIdx.x;
  double loss = 0.0;
  if (ACCALL) {
    if (line >= a.lines) return;
    float2 sum[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) sum[r] = make_float2(0.0f, 0.0f);
    for (int img = 0; img < a.n_acc; ++img) {
      float2 v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = make_float2(0.0f, 0.0f);
      load_pre<N, 1>(a, img, line * N, v);
      dft<N, DIR>(v);
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const float2 h = a.H[(long long)img * a.H_stride + line * N + r];
        sum[r] = cadd(sum[r], cmul(conjf2(h), make_float2(v[r].x * a.scale, v[r].y * a.scale)));
      }
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const long long p = line * N + r;
      a.acc[p] = a.accumulate ? cadd(a.acc[p], sum[r]) : sum[r];
    }
    return;
  }
  const int img = blockIdx.y;
  if (line < a.lines) {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = make_float2(0.0f, 0.0f);
    load_pre<N, 1>(a, img, line * N, v);
    dft<N, DIR>(v);
    int pos[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) pos[r] = r;
    post_block<N>(a, img, line * N, pos, v, loss);
  }
  if (a.post == kPostResidual) {
    const double tot = block_sum(loss, red);
    if (threadIdx.x == 0) a.partial[(long long)img * gridDim.x + blockIdx.x] = tot;
  }
}

// Column pass: input image [N][W] (W = a.lines columns, rows contiguous), an
// FFT along every N-long column, column c written as line c of the output, so
// the output image is the transposed [W][N] - a line pass fused with the
// transpose. CB columns per block are staged through LDS with row-contiguous
// loads (CB * 8 bytes per row); the radix passes then run as in line_fft and
// each column's result is stored as one contiguous line. Same epilogues as the
// line kernel, indexed in the output layout (no pre-multiply, no
// accumulate-all). 8 columns per block (two blocks per CU at N = 1024)
// measured faster than 16 (one block per CU) or 4 (32-byte row segments) when
// there are blocks for every CU; a single image of fewer than 2048 columns
// gives fewer, and then 4 columns per block spread it over twice the CUs.
template <int N>
constexpr int col_block() { return (512 / (N / 16)) < 8 ? (512 / (N / 16)) : 8; }

// Stage the CB columns of group grp of an [N][W] image into LDS (column c at
// s + c * LS, pidx positions) with row-contiguous loads: the 16 loads of a thread are all issued
// before the first LDS write, so they are in flight together (N * CB = 16 NT).
// A thread's column is the same for all 16 (NT is a multiple of CB) and its
// rows are row0 + k * TPL; past the last column it loads column W - 1 and
// stages zeros, so that no load sits in a branch of its own (which would make
// each wait for the previous one). Offsets within an image are 32-bit (the
// launchers check N * W < 2^31), one register per address.
template <int N, int CB, int NT, int LS, int E = 16>
__device__ __forceinline__ void stage_columns(const float2* __restrict__ in, int W, int grp, float2* s) {
  static_assert(N * CB == E * NT && NT % CB == 0, "E elements per thread, one column per thread");
  constexpr int RSTEP = NT / CB;  // rows between a thread's consecutive elements
  const int c = threadIdx.x % CB, row0 = threadIdx.x / CB;
  const int gc = grp * CB + c;
  const bool in_range = gc < W;
  const int base = row0 * W + (in_range ? gc : W - 1);
  float2 v[16];
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = in[base + k * RSTEP * W];
#pragma unroll
  for (int k = 0; k < E; ++k)
    if (!in_range) v[k] = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int k = 0; k < E; ++k) s[c * LS + pidx(row0 + k * RSTEP)] = v[k];
  __syncthreads();
}

// The inverse of stage_columns: CB staged columns back to an [N][W] image
// with row-contiguous stores (columns past W are not written).
template <int N, int CB, int NT, int LS>
__device__ __forceinline__ void unstage_columns(const float2* s, int W, int grp, float2* __restrict__ out) {
  constexpr int RSTEP = NT / CB;
  const int c = threadIdx.x % CB, row0 = threadIdx.x / CB;
  const int gc = grp * CB + c;
  float2 v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = s[c * LS + pidx(row0 + k * RSTEP)];
  if (gc < W) {
    const int base = row0 * W + gc;
#pragma unroll
    for (int k = 0; k < 16; ++k) out[base + k * RSTEP * W] = v[k];
  }
}

template <int N, int DIR, int CB, int E = 16>
__global__ __launch_bounds__(CB * (N / E)) void fft_col_kernel(FftArgs a) {
  constexpr int TPL = N / E;
  constexpr int NT = CB * TPL;
  // padded line: with a pitch of 4 (mod 32) elements beyond the pidx length the
  // column-staging accesses (CB columns x consecutive rows per wave) measured the
  // fewest LDS bank conflicts (pitches +0, +1, +8, +17 had 1.1-3x as many)
  constexpr int LS = N + N / 16 + 4;
  __shared__ float2 s[CB * LS];
  __shared__ float2 twh[N / 2];
  __shared__ double red[(NT + 63) / 64];
  const long long W = a.lines;
  const int cl = threadIdx.x / TPL;
  const int grp = xcd_remap(blockIdx.x, gridDim.x);  // neighbouring column groups share an L2
  const long long col = (long long)grp * CB + cl;
  const bool live = col < W;
  float2* sl = s + cl * LS;
  const int img = blockIdx.y;
  TwStage<N, NT> tws;
  tws.fetch(a.tw);
  stage_columns<N, CB, NT, LS, E>(a.in + (long long)img * a.in_stride, (int)W, grp, s);
  tws.store(twh);
  float2 o[16], v[16];
  int pos[16];
  line_from_lds<N, E>(sl, v);
  line_fft_regs<N, DIR, false, E>(sl, twh, v, o, pos);
  double loss = 0.0;
  if (live) post_block<E>(a, img, col * N, pos, o, loss);
  if (a.post == kPostResidual) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (NT + 63) / 64; ++w) t += red[w];
      a.partial[(long long)img * gridDim.x + blockIdx.x] = t;
    }
  }
}

// Round trip along the columns of an [N][W] image (the transposed spectrum
// layout: N = n, W = m), for the gradient of Eq. (27): the inverse DFT of every
// column (which completes A_d x, the m-direction having been inverted by the
// previous pass), the residual bracket (A x / |A x|)(|A x| - sqrt(y)) in the
// spatial domain (with float64 loss partials), and the forward DFT of that
// column again, stored back in the same [N][W] layout - no transpose, and the
// residual never goes to memory. Column c of the image is row c of the
// natural-layout image, so sqrt(y) is read at c * N + k. Columns are staged
// through LDS for row-contiguous loads and stores, as in fft_col_kernel.
// Two blocks share a CU where the LDS fits two (N <= 2048), so at most 128
// VGPRs per lane there.
template <int N>
__global__ __launch_bounds__(col_block<N>() * (N / 16)) __attribute__((amdgpu_waves_per_eu(N <= 2048 ? 4 : 2)))
void fft_col_roundtrip_kernel(FftArgs a) {
  constexpr int TPL = N / 16;
  constexpr int CB = col_block<N>();
  constexpr int NT = CB * TPL;
  constexpr int LS = N + N / 16 + 4;  // as in fft_col_kernel
  __shared__ float2 s[CB * LS];
  __shared__ float2 twh[N / 2];
  __shared__ double red[(NT + 63) / 64];
  const long long W = a.lines;
  const int cl = threadIdx.x / TPL;
  const int grp = xcd_remap(blockIdx.x, gridDim.x);  // neighbouring column groups share an L2
  const long long col = (long long)grp * CB + cl;
  const bool live = col < W;
  float2* sl = s + cl * LS;
  const int img = blockIdx.y;
  TwStage<N, NT> tws;
  tws.fetch(a.tw);
  stage_columns<N, CB, NT, LS>(a.in + (long long)img * a.in_stride, (int)W, grp, s);
  tws.store(twh);
  float2 o[16];
  int pos[16];
  {
    float2 v[16];
    line_from_lds<N>(sl, v);
    line_fft_regs<N, 1>(sl, twh, v, o, pos);
  }
  __syncthreads();  // every thread's last inverse pass has read its line
#pragma unroll
  for (int r = 0; r < 16; ++r) sl[pidx(pos[r])] = o[r];
  __syncthreads();
  // the residual at the positions lt + r * TPL, which are the inputs of this
  // thread's first forward pass: the forward transform starts from registers
  const int lt = threadIdx.x % TPL;
  const float* sy = a.sy + (long long)img * a.sy_stride + (live ? col : 0) * N + lt;
  float y[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) y[r] = sy[r * TPL];
  float2 v[16];
  double loss = 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float2 w = sl[pidx(lt + r * TPL)];
    const float2 u = make_float2(w.x * a.scale, w.y * a.scale);
    const float am = sqrtf(u.x * u.x + u.y * u.y);
    const float res = am - (live ? y[r] : 0.0f);
    float2 ph = make_float2(1.0f, 0.0f);
    if (am > 0.0f) ph = make_float2(u.x / am, u.y / am);
    v[r] = make_float2(ph.x * res, ph.y * res);
    if (live) loss += 0.5 * (double)res * (double)res;
  }
  line_fft_regs<N, -1, true>(sl, twh, v, o, pos);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) sl[pidx(pos[r])] = o[r];
  __syncthreads();
  unstage_columns<N, CB, NT, LS>(s, (int)W, grp, a.out + (long long)img * a.img_stride);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (NT + 63) / 64; ++w) t += red[w];
    a.partial[(long long)img * gridDim.x + blockIdx.x] = t;
  }
}

// out[c][r] = in[r][c] for an R x C complex array per image, 64 x 64 tiles.
__global__ __launch_bounds__(kThreads) void transpose_kernel(const float2* __restrict__ in, float2* __restrict__ out,
                                                              int R, int C, long long stride) {
  __shared__ float2 t[64][65];
  const int tilesC = (C + 63) / 64;
  const int tile = blockIdx.x;
  const int tr = tile / tilesC, tc = tile - tr * tilesC;
  const float2* src = in + (long long)blockIdx.y * stride;
  float2* dst = out + (long long)blockIdx.y * stride;
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = tr * 64 + ly + 4 * i, c = tc * 64 + lx;
    if (r < R && c < C) t[ly + 4 * i][lx] = src[(long long)r * C + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int c = tc * 64 + ly + 4 * i, r = tr * 64 + lx;
    if (r < R && c < C) dst[(long long)c * R + r] = t[lx][ly + 4 * i];
  }
}

__global__ __launch_bounds__(256) void twiddle_kernel(float2* tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double sn, cs;
  sincospi(-2.0 * (double)k / (double)N, &sn, &cs);
  tw[k] = make_float2((float)cs, (float)sn);
}

// H_d(f_x, f_y) of Eq. (23) on the unshifted FFT frequency grid (numpy's fftfreq
// order), zero on the evanescent band, stored transposed: H_t[j][i] for row
// frequency index i (of m) and column frequency index j (of n).
__global__ __launch_bounds__(256) void transfer_t_kernel(float2* Ht, int m, int n, double dist, double wavelength,
                                                         double pixel) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)m * n) return;
  const int j = (int)(p / m), i = (int)(p - (long long)j * m);
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
  Ht[p] = h;
}

__global__ __launch_bounds__(256) void sqrt_y_kernel(const float* __restrict__ y, float* __restrict__ sy,
                                                     float2* __restrict__ syc, long long total) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const float v = sqrtf(fmaxf(y[p], 0.0f));
  sy[p] = v;
  if (syc) syc[p] = make_float2(v, 0.0f);
}

// Sum of partial[i * stride + j] over i < count by one wave: lane l adds the
// terms l, l + 64, ... in order, then a fixed butterfly combines the lanes,
// so the summation order (and the result) is the same on every run.
__device__ __forceinline__ double wave_sum_strided(const double* __restrict__ partial, int count,
                                                   long long stride, int j) {
  double s = 0.0;
  for (int i = (int)threadIdx.x; i < count; i += 64) s += partial[(long long)i * stride + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

__global__ __launch_bounds__(64) void loss_final_kernel(const double* __restrict__ partial, int count,
                                                        float* __restrict__ out) {
  const double s = wave_sum_strided(partial, count, 1, 0);
  if (threadIdx.x == 0) *out = (float)s;
}

// out[j] = sum_i partial[i * stride + j] for j < width (one wave per j; deterministic).
__global__ __launch_bounds__(64) void sum_d_kernel(const double* __restrict__ partial, int count, int stride,
                                                   int width, double* __restrict__ out) {
  const int j = blockIdx.x;
  const double s = wave_sum_strided(partial, count, stride, j);
  if (threadIdx.x == 0 && j < width) out[j] = s;
}

__global__ __launch_bounds__(256) void fill_f32_kernel(float* __restrict__ p, float v, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// v = z - gamma g (the argument of Algorithm 1's prox).
__global__ __launch_bounds__(256) void grad_step_kernel(const float2* __restrict__ z, const float2* __restrict__ g,
                                                        float gamma, float2* __restrict__ v, long long total) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const float2 zv = z[p], gv = g[p];
  v[p] = make_float2(fmaf(-gamma, gv.x, zv.x), fmaf(-gamma, gv.y, zv.y));
}

// Per-block partials of Re<g, x - z> and ||x - z||^2 in float64 (the two
// inner products of the backtracking test), [block][2].
__global__ __launch_bounds__(256) void ls_dots_kernel(const float2* __restrict__ g, const float2* __restrict__ x,
                                                      const float2* __restrict__ z, long long total,
                                                      double* __restrict__ partial) {
  __shared__ double red[2][4];
  double a = 0.0, q = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (long long)gridDim.x * blockDim.x) {
    const float2 gv = g[p], xv = x[p], zv = z[p];
    const double dx = (double)xv.x - (double)zv.x, dy = (double)xv.y - (double)zv.y;
    a += (double)gv.x * dx + (double)gv.y * dy;
    q += dx * dx + dy * dy;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    q += __shfl_xor(q, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    partial[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(256) void copy_c_kernel(const float2* __restrict__ a, float2* __restrict__ b,
                                                     long long total) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < total) b[p] = a[p];
}

// A pass of `lines` N-point lines (all images) gives fewer than 8 waves per
// CU at 16 elements per thread: run it at 8 (256 <= N <= 2048).
bool fft_few_waves(int N, long long lines) {
  return N >= 256 && N <= 2048 && lines * (long long)N < (1LL << 21);
}

template <int DIR, bool ACCALL>
hipError_t launch_line_dir(const FftArgs& a, int N, int batch, hipStream_t s) {
  const long long lines = a.lines;
  if (N <= 16) {
    const dim3 grid((unsigned)((lines + kThreads - 1) / kThreads), (unsigned)batch);
    switch (N) {
      case 2: hipLaunchKernelGGL((fft_small_kernel<2, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
      case 4: hipLaunchKernelGGL((fft_small_kernel<4, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
      case 8: hipLaunchKernelGGL((fft_small_kernel<8, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
      default: hipLaunchKernelGGL((fft_small_kernel<16, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    }
    return hipGetLastError();
  }
  if (!ACCALL && fft_few_waves(N, lines * batch)) {
    // 8 elements per thread: twice the threads per line for a pass that would
    // otherwise leave each CU a handful of waves
    const int lpb8 = kThreads / (N / 8);
    const dim3 grid8((unsigned)((lines + lpb8 - 1) / lpb8), (unsigned)batch);
    switch (N) {
      case 256: hipLaunchKernelGGL((fft_line_kernel<256, DIR, false, 8>), grid8, dim3(kThreads), 0, s, a); break;
      case 512: hipLaunchKernelGGL((fft_line_kernel<512, DIR, false, 8>), grid8, dim3(kThreads), 0, s, a); break;
      case 1024: hipLaunchKernelGGL((fft_line_kernel<1024, DIR, false, 8>), grid8, dim3(kThreads), 0, s, a); break;
      default: hipLaunchKernelGGL((fft_line_kernel<2048, DIR, false, 8>), grid8, dim3(kThreads), 0, s, a); break;
    }
    return hipGetLastError();
  }
  const int lpb = kThreads / (N / 16);
  const dim3 grid((unsigned)((lines + lpb - 1) / lpb), (unsigned)batch);
  switch (N) {
    case 32: hipLaunchKernelGGL((fft_line_kernel<32, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    case 64: hipLaunchKernelGGL((fft_line_kernel<64, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    case 128: hipLaunchKernelGGL((fft_line_kernel<128, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    case 256: hipLaunchKernelGGL((fft_line_kernel<256, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    case 512: hipLaunchKernelGGL((fft_line_kernel<512, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    case 1024: hipLaunchKernelGGL((fft_line_kernel<1024, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    case 2048: hipLaunchKernelGGL((fft_line_kernel<2048, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((fft_line_kernel<4096, DIR, ACCALL>), grid, dim3(kThreads), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace

bool fft_size_ok(int v) { return v >= 2 && v <= 4096 && (v & (v - 1)) == 0; }

int fft_line_blocks(int N, long long lines) {
  if (N <= 16) return (int)((lines + kThreads - 1) / kThreads);
  const int lpb = kThreads / (N / 16);
  return (int)((lines + lpb - 1) / lpb);
}

hipError_t launch_fft_lines(FftArgs a, int N, long long lines, int dir, int batch, hipStream_t s) {
  a.lines = lines;
  if (a.post == kPostAccumulateAll)  // the images are looped inside the kernel
    return dir < 0 ? launch_line_dir<-1, true>(a, N, 1, s) : launch_line_dir<1, true>(a, N, 1, s);
  return dir < 0 ? launch_line_dir<-1, false>(a, N, batch, s) : launch_line_dir<1, false>(a, N, batch, s);
}

template <int DIR>
static hipError_t launch_col_dir(const FftArgs& a, int N, int batch, hipStream_t s) {
  // 4 columns per block where 8 would leave CUs idle (not for the residual
  // epilogue, whose loss partials are counted per 8-column block)
  const bool narrow = a.post != kPostResidual && (a.lines + 7) / 8 * batch < 256;
  // 8 elements per thread where 16 would leave each CU a handful of waves
  const bool e8 = fft_few_waves(N, a.lines * batch);
#define CTV_COLK(NN)                                                                        \
  case NN: {                                                                                \
    constexpr int cb = col_block<NN>();                                                     \
    constexpr int cbn = cb == 8 && NN >= 256 ? 4 : cb;                                      \
    constexpr int e8ok = NN >= 256 && NN <= 2048;                                           \
    if (narrow && cbn != cb) {                                                              \
      const dim3 grid((unsigned)((a.lines + cbn - 1) / cbn), (unsigned)batch);             \
      if (e8ok && e8)                                                                       \
        hipLaunchKernelGGL((fft_col_kernel<NN, DIR, cbn, e8ok ? 8 : 16>), grid, dim3(cbn * (NN / (e8ok ? 8 : 16))), 0, s, a); \
      else                                                                                  \
        hipLaunchKernelGGL((fft_col_kernel<NN, DIR, cbn>), grid, dim3(cbn * (NN / 16)), 0, s, a); \
    } else {                                                                                \
      const dim3 grid((unsigned)((a.lines + cb - 1) / cb), (unsigned)batch);                \
      if (e8ok && e8)                                                                       \
        hipLaunchKernelGGL((fft_col_kernel<NN, DIR, cb, e8ok ? 8 : 16>), grid, dim3(cb * (NN / (e8ok ? 8 : 16))), 0, s, a); \
      else                                                                                  \
        hipLaunchKernelGGL((fft_col_kernel<NN, DIR, cb>), grid, dim3(cb * (NN / 16)), 0, s, a); \
    }                                                                                       \
    break;                                                                                  \
  }
  switch (N) {
    CTV_COLK(32) CTV_COLK(64) CTV_COLK(128) CTV_COLK(256) CTV_COLK(512) CTV_COLK(1024) CTV_COLK(2048) CTV_COLK(4096)
    default: return hipErrorInvalidValue;
  }
#undef CTV_COLK
  return hipGetLastError();
}

int fft_second_blocks(int N, long long W) {
  if (N <= 16) return fft_line_blocks(N, W);
  const int cb = (512 / (N / 16)) < 8 ? (512 / (N / 16)) : 8;  // col_block<N>
  return (int)((W + cb - 1) / cb);
}

hipError_t launch_fft_second(FftArgs a, int N, long long W, int dir, int batch, float2* tmp, hipStream_t s) {
  if (N <= 16 || a.post == kPostAccumulateAll) {
    // transpose into tmp, then a line pass with the same epilogue: short
    // columns, and the accumulate-all epilogue (its images are looped inside
    // one block, which measured faster on line blocks than on staged columns)
    hipError_t e = launch_transpose(a.in, tmp, N, (int)W, a.post == kPostAccumulateAll ? a.n_acc : batch, s);
    if (e != hipSuccess) return e;
    a.in = tmp;
    return launch_fft_lines(a, N, W, dir, batch, s);
  }
  if (a.pre != kPreNone) return hipErrorInvalidValue;
  if ((long long)N * W > INT_MAX) return hipErrorInvalidValue;  // 32-bit offsets within an image
  a.lines = W;
  return dir < 0 ? launch_col_dir<-1>(a, N, batch, s) : launch_col_dir<1>(a, N, batch, s);
}

hipError_t launch_fft_roundtrip(FftArgs a, int N, long long W, int batch, hipStream_t s) {
  if ((long long)N * W > INT_MAX) return hipErrorInvalidValue;  // 32-bit offsets within an image
  a.lines = W;
#define CTV_RTK(NN)                                                                            \
  case NN: {                                                                                   \
    constexpr int cb = col_block<NN>();                                                        \
    const dim3 grid((unsigned)((W + cb - 1) / cb), (unsigned)batch);                           \
    hipLaunchKernelGGL((fft_col_roundtrip_kernel<NN>), grid, dim3(cb * (NN / 16)), 0, s, a);   \
    break;                                                                                     \
  }
  switch (N) {
    CTV_RTK(32) CTV_RTK(64) CTV_RTK(128) CTV_RTK(256) CTV_RTK(512) CTV_RTK(1024) CTV_RTK(2048) CTV_RTK(4096)
    default: return hipErrorInvalidValue;
  }
#undef CTV_RTK
  return hipGetLastError();
}

hipError_t launch_fft_acc_inverse(FftArgs a, int N, long long lines, hipStream_t s) {
  a.lines = lines;
#define CTV_AIK(NN)                                                                     \
  case NN: {                                                                            \
    constexpr int lpb = acc_lines_per_block<NN>();                                      \
    const dim3 grid((unsigned)((lines + lpb - 1) / lpb));                               \
    if (a.n_acc <= acc_groups<NN>())                                                    \
      hipLaunchKernelGGL((fft_acc_inverse_kernel<NN, true>), grid, dim3(kThreads), 0, s, a); \
    else                                                                                \
      hipLaunchKernelGGL((fft_acc_inverse_kernel<NN, false>), grid, dim3(kThreads), 0, s, a); \
    break;                                                                              \
  }
  switch (N) {
    CTV_AIK(32) CTV_AIK(64) CTV_AIK(128) CTV_AIK(256) CTV_AIK(512) CTV_AIK(1024) CTV_AIK(2048) CTV_AIK(4096)
    default: return hipErrorInvalidValue;
  }
#undef CTV_AIK
  return hipGetLastError();
}

hipError_t launch_transpose(const float2* in, float2* out, int R, int C, int batch, hipStream_t s) {
  const int tiles = ((R + 63) / 64) * ((C + 63) / 64);
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)tiles, (unsigned)batch), dim3(kThreads), 0, s, in, out, R, C,
                     (long long)R * C);
  return hipGetLastError();
}

hipError_t launch_twiddles(float2* tw, int N, hipStream_t s) {
  hipLaunchKernelGGL(twiddle_kernel, dim3((N + 255) / 256), dim3(256), 0, s, tw, N);
  return hipGetLastError();
}

hipError_t launch_transfer_t(float2* Ht, int m, int n, double dist, double wavelength, double pixel, hipStream_t s) {
  const long long total = (long long)m * n;
  hipLaunchKernelGGL(transfer_t_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Ht, m, n, dist,
                     wavelength, pixel);
  return hipGetLastError();
}

hipError_t launch_sqrt_y(const float* y, float* sy, float2* syc, long long total, hipStream_t s) {
  hipLaunchKernelGGL(sqrt_y_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, y, sy, syc, total);
  return hipGetLastError();
}

hipError_t launch_loss_final(const double* partial, int count, float* out, hipStream_t s) {
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, partial, count, out);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, long long count, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_sum_d(const double* partial, int count, int stride, int width, double* out, hipStream_t s) {
  if (width < 1) return hipSuccess;
  hipLaunchKernelGGL(sum_d_kernel, dim3((unsigned)width), dim3(64), 0, s, partial, count, stride, width, out);
  return hipGetLastError();
}

hipError_t launch_grad_step(const float2* z, const float2* g, float gamma, float2* v, long long total, hipStream_t s) {
  hipLaunchKernelGGL(grad_step_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, z, g, gamma, v, total);
  return hipGetLastError();
}

hipError_t launch_ls_dots(const float2* g, const float2* x, const float2* z, long long total, double* partial,
                          hipStream_t s) {
  hipLaunchKernelGGL(ls_dots_kernel, dim3(kLsBlocks), dim3(256), 0, s, g, x, z, total, partial);
  return hipGetLastError();
}

hipError_t launch_copy_c(const float2* a, float2* b, long long total, hipStream_t s) {
  hipLaunchKernelGGL(copy_c_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, b, total);
  return hipGetLastError();
}

}  // namespace ctv
