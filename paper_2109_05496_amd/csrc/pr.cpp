// Host side of the phase-retrieval path: FISTA (Algorithm 1) on the amplitude
// data term of Eq. (24) summed over the measurement distances, with the
// constrained-TV FGP denoiser as the proximity operator (Eq. 15, lambda =
// tau * gamma), plus the stage entry points and the standalone 2-D FFT.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctv.h"
#include "ctv_host.hpp"
#include "ctv_pr.hpp"

using namespace ctv;

namespace {

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct PrLayout {
  size_t tw_n, tw_m, H, sy, syc, xh, t1, t2, acc, v, xcur, xprev, z, fgp, part, g, warm, lsp, lsv, total;
};

// Blocks of the residual pass (the second pass of an inverse transform: columns of length n, m of them).
int residual_blocks(int m, int n) { return fft_second_blocks(n, m); }

PrLayout pr_layout(int D, int m, int n) {
  PrLayout L;
  const size_t px = (size_t)m * n;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.tw_n = take((size_t)n * 8);
  L.tw_m = take((size_t)m * 8);
  L.H = take((size_t)D * px * 8);  // transposed transfer functions [D][n][m]
  L.sy = take((size_t)D * px * 4);
  L.syc = take((size_t)D * px * 8);
  L.xh = take(px * 8);
  L.t1 = take((size_t)D * px * 8);  // per-distance temporaries
  L.t2 = take((size_t)D * px * 8);
  L.acc = take(px * 8);
  L.v = take(px * 8);
  L.xcur = take(px * 8);
  L.xprev = take(px * 8);
  L.z = take(px * 8);
  L.fgp = take(denoise_ws_bytes(1, m, n));
  L.part = take((size_t)D * residual_blocks(m, n) * 8);
  L.g = take(px * 8);                              // grad F(z) (line search)
  L.warm = take(2 * align_up(state_bytes(1, m, n)));  // warm-start dual: current, next
  L.lsp = take((size_t)kLsBlocks * 2 * 8);          // inner-product partials
  L.lsv = take(4 * 8);                              // F(z), F(x), Re<g, x - z>, ||x - z||^2
  L.total = o;
  return L;
}

ctv_status validate_pr(const pr_params* p, int m, int n, bool need_inner) {
  if (!p) return fail(CTV_ERR_INVALID_ARG, "pr_params is NULL");
  if (p->struct_size != sizeof(pr_params)) return fail(CTV_ERR_INVALID_ARG, "pr_params.struct_size mismatch");
  if (p->num_meas < 1 || p->num_meas > 64) return fail(CTV_ERR_INVALID_ARG, "num_meas must lie in [1, 64]");
  if (!p->distances_host) return fail(CTV_ERR_INVALID_ARG, "distances_host is NULL");
  for (int d = 0; d < p->num_meas; ++d)
    if (!std::isfinite(p->distances_host[d])) return fail(CTV_ERR_INVALID_ARG, "non-finite distance");
  if (!(p->wavelength > 0.0) || !std::isfinite(p->wavelength)) return fail(CTV_ERR_INVALID_ARG, "wavelength must be > 0");
  if (!(p->pixel > 0.0) || !std::isfinite(p->pixel)) return fail(CTV_ERR_INVALID_ARG, "pixel must be > 0");
  if (!fft_size_ok(m) || !fft_size_ok(n)) return fail(CTV_ERR_UNSUPPORTED, "m and n must be powers of two in [2, 4096]");
  if (need_inner) {
    if (!(p->tau >= 0.0f) || !std::isfinite(p->tau)) return fail(CTV_ERR_INVALID_ARG, "tau must be >= 0");
    if (!(p->gamma >= 0.0f) || !std::isfinite(p->gamma)) return fail(CTV_ERR_INVALID_ARG, "gamma must be >= 0");
    const double g0 = p->gamma > 0.0f ? (double)p->gamma : 1.0 / p->num_meas;
    if (p->tau > 0.0f && (double)p->tau * g0 < (double)kMinLambda)
      return fail(CTV_ERR_INVALID_ARG, "tau * gamma must be 0 or >= 1e-12 (the prox's lambda)");
    if (p->outer_iters < 0) return fail(CTV_ERR_INVALID_ARG, "outer_iters must be >= 0");
    ctv_status st = validate_params(&p->inner);
    if (st) return st;
    if (p->line_search) {
      if (!(p->ls_shrink > 0.0f && p->ls_shrink < 1.0f)) return fail(CTV_ERR_INVALID_ARG, "ls_shrink must lie in (0, 1)");
      if (p->ls_max_trials < 1) return fail(CTV_ERR_INVALID_ARG, "ls_max_trials must be >= 1");
    }
  }
  return CTV_OK;
}

#define CTV_TRY(expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, what);   \
  } while (0)

struct Ctx {
  int m, n, D;
  long long px;
  char* ws;
  PrLayout L;
  hipStream_t s;
  float2* at(size_t off) const { return reinterpret_cast<float2*>(ws + off); }
  float* atf(size_t off) const { return reinterpret_cast<float*>(ws + off); }
  const float2* Ht(int d) const { return at(L.H) + (size_t)d * px; }
  const float* sy(int d) const { return atf(L.sy) + (size_t)d * px; }
};

FftArgs line_args(const float2* in, float2* out, const float2* tw, long long stride) {
  FftArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.tw = tw;
  a.in_stride = stride;
  a.img_stride = stride;
  a.scale = 1.0f;
  a.pre = kPreNone;
  a.post = kPostStore;
  return a;
}

// Spectrum (transposed, [n][m]) of a natural-layout [m][n] image: a pass along
// n, then a column pass along m that writes the transposed layout, with
// epilogue `last` (in/out/tw filled here).
// The momentum step of Algorithm 1 (line 5) done in the first pass of the
// next transform: z = x + beta (x - x_prev), stored to z on the way.
struct Extrapolate {
  const float2* x_prev;
  float beta;
  float2* z;
};

ctv_status fft2_to_t(const Ctx& c, const float2* in, float2* out, FftArgs last, const Extrapolate* ex = nullptr) {
  float2* t1 = c.at(c.L.t1);
  float2* t2 = c.at(c.L.t2);
  FftArgs a = line_args(in, t1, c.at(c.L.tw_n), c.px);
  if (ex) {
    a.pre = kPreExtrapolate;
    a.in2 = ex->x_prev;
    a.beta = ex->beta;
    a.zout = ex->z;
  }
  CTV_TRY(launch_fft_lines(a, c.n, c.m, -1, 1, c.s), "fft (rows)");
  last.in = t1;
  last.out = out;
  last.tw = c.at(c.L.tw_m);
  last.in_stride = last.img_stride = c.px;
  CTV_TRY(launch_fft_second(last, c.m, c.n, -1, 1, t2, c.s), "fft (columns)");
  return CTV_OK;
}

// Inverse transform of a transposed spectrum [n][m] to natural layout [m][n]:
// a pass along m (optionally multiplying by Ht on load), then a column pass
// along n that writes the natural layout, with epilogue `last` (scale 1/(mn)
// folded in by the caller).
ctv_status ifft2_from_t(const Ctx& c, const float2* in, const float2* Ht, float2* out, FftArgs last,
                        int pre = kPreMulH) {
  float2* t1 = c.at(c.L.t1);
  float2* t2 = c.at(c.L.t2);
  FftArgs a = line_args(in, t1, c.at(c.L.tw_m), c.px);
  if (Ht) {
    a.pre = pre;
    a.H = Ht;
  }
  CTV_TRY(launch_fft_lines(a, c.m, c.n, 1, 1, c.s), "ifft (columns)");
  last.in = t1;
  last.out = out;
  last.tw = c.at(c.L.tw_n);
  last.in_stride = last.img_stride = c.px;
  CTV_TRY(launch_fft_second(last, c.n, c.m, 1, 1, t2, c.s), "ifft (rows)");
  return CTV_OK;
}

FftArgs epilogue(int post, float scale) {
  FftArgs a = line_args(nullptr, nullptr, nullptr, 0);
  a.post = post;
  a.scale = scale;
  return a;
}

// Tables shared by every phase-retrieval entry point: twiddles, H_d (transposed), sqrt(y_d).
ctv_status build_tables(const Ctx& c, const pr_params* p, const float* y) {
  CTV_TRY(launch_twiddles(c.at(c.L.tw_n), c.n, c.s), "twiddles");
  CTV_TRY(launch_twiddles(c.at(c.L.tw_m), c.m, c.s), "twiddles");
  for (int d = 0; d < c.D; ++d)
    CTV_TRY(launch_transfer_t(c.at(c.L.H) + (size_t)d * c.px, c.m, c.n, p->distances_host[d], p->wavelength,
                              p->pixel, c.s), "transfer function");
  if (y) CTV_TRY(launch_sqrt_y(y, c.atf(c.L.sy), nullptr, (long long)c.D * c.px, c.s), "sqrt(y)");
  return CTV_OK;
}

// For every distance at once (batch D): the transposed spectra
// conj(H_d) * FFT2(r_d) of the natural-layout images r_d (stride px), summed
// over d into acc inside the last pass.
ctv_status accumulate_spectra(const Ctx& c, const float2* r, float2* acc) {
  float2* t1 = c.at(c.L.t1);
  float2* t2 = c.at(c.L.t2);
  CTV_TRY(launch_fft_lines(line_args(r, t1, c.at(c.L.tw_n), c.px), c.n, c.m, -1, c.D, c.s), "fft (rows)");
  FftArgs q = line_args(t1, nullptr, c.at(c.L.tw_m), c.px);
  q.post = kPostAccumulateAll;
  q.H = c.Ht(0);
  q.H_stride = c.px;
  q.acc = acc;
  q.accumulate = 0;
  q.n_acc = c.D;
  CTV_TRY(launch_fft_second(q, c.m, c.n, -1, 1, t2, c.s), "fft (columns, accumulate)");
  return CTV_OK;
}

// grad F at z (Eq. 27 summed over d). post_step: out = z - gamma grad; else out = grad.
// With ex, z is first formed from the two latest iterates (z given as x, ex->z
// receives it).
ctv_status gradient(const Ctx& c, const float2* z, float2* out, bool post_step, float gamma, float* loss,
                    const Extrapolate* ex = nullptr) {
  const float inv = 1.0f / (float)((double)c.m * c.n);
  float2* xh = c.at(c.L.xh);
  float2* t1 = c.at(c.L.t1);
  float2* t2 = c.at(c.L.t2);
  float2* acc = c.at(c.L.acc);
  double* part = reinterpret_cast<double*>(c.ws + c.L.part);
  const int rb = residual_blocks(c.m, c.n);
  ctv_status st = fft2_to_t(c, z, xh, epilogue(kPostStore, 1.0f), ex);
  if (st) return st;
  if (ex) z = ex->z;
  // A_d z = IFFT2(H_d Z) for all d (one shared input spectrum), then the
  // residual bracket of Eq. (27) in t2[d]
  FftArgs a = line_args(xh, t1, c.at(c.L.tw_m), c.px);
  a.in_stride = 0;
  a.pre = kPreMulH;
  a.H = c.Ht(0);
  a.H_stride = c.px;
  CTV_TRY(launch_fft_lines(a, c.m, c.n, 1, c.D, c.s), "ifft (columns)");
  if (c.n >= 32) {
    // along n: inverse, residual, forward again in one pass (t1 -> t2, [n][m]);
    // then the forward pass along m with acc = sum_d conj(H_d) (.) over the distances
    FftArgs r = line_args(t1, t2, c.at(c.L.tw_n), c.px);
    r.scale = inv;
    r.sy = c.sy(0);
    r.sy_stride = c.px;
    r.partial = part;
    CTV_TRY(launch_fft_roundtrip(r, c.n, c.m, c.D, c.s), "residual round trip");
    if (c.m >= 32) {
      // along m: forward, sum_d conj(H_d) (.) over the distances, inverse of the
      // sum (t2 -> t1, [n][m]); then the inverse along n with the epilogue
      FftArgs q = line_args(t2, t1, c.at(c.L.tw_m), c.px);
      q.H = c.Ht(0);
      q.H_stride = c.px;
      q.n_acc = c.D;
      CTV_TRY(launch_fft_acc_inverse(q, c.m, c.n, c.s), "fft (columns, accumulate, inverse)");
      FftArgs g = epilogue(post_step ? kPostStep : kPostStore, inv);
      g.z = z;
      g.gamma = gamma;
      g.in = t1;
      g.out = out;
      g.tw = c.at(c.L.tw_n);
      g.in_stride = g.img_stride = c.px;
      CTV_TRY(launch_fft_second(g, c.n, c.m, 1, 1, t2, c.s), "ifft (rows)");
      if (loss) CTV_TRY(launch_loss_final(part, c.D * rb, loss, c.s), "loss");
      return CTV_OK;
    }
    FftArgs q = line_args(t2, nullptr, c.at(c.L.tw_m), c.px);
    q.post = kPostAccumulateAll;
    q.H = c.Ht(0);
    q.H_stride = c.px;
    q.acc = acc;
    q.accumulate = 0;
    q.n_acc = c.D;
    CTV_TRY(launch_fft_lines(q, c.m, c.n, -1, 1, c.s), "fft (columns, accumulate)");
  } else {
    FftArgs r = line_args(t1, t2, c.at(c.L.tw_n), c.px);
    r.post = kPostResidual;
    r.scale = inv;
    r.sy = c.sy(0);
    r.sy_stride = c.px;
    r.partial = part;
    CTV_TRY(launch_fft_second(r, c.n, c.m, 1, c.D, t2, c.s), "ifft (rows, residual)");
    // acc = sum_d conj(H_d) FFT2(residual_d)
    st = accumulate_spectra(c, t2, acc);
    if (st) return st;
  }
  FftArgs g = epilogue(post_step ? kPostStep : kPostStore, inv);
  g.z = z;
  g.gamma = gamma;
  st = ifft2_from_t(c, acc, nullptr, out, g);
  if (st) return st;
  if (loss) CTV_TRY(launch_loss_final(part, c.D * rb, loss, c.s), "loss");
  return CTV_OK;
}

// F(x) (Eq. 24 summed over d) into *out (device double): the forward half of gradient().
ctv_status data_term(const Ctx& c, const float2* x, double* out) {
  float2* xh = c.at(c.L.xh);
  float2* t1 = c.at(c.L.t1);
  float2* t2 = c.at(c.L.t2);
  double* part = reinterpret_cast<double*>(c.ws + c.L.part);
  ctv_status st = fft2_to_t(c, x, xh, epilogue(kPostStore, 1.0f));
  if (st) return st;
  FftArgs a = line_args(xh, t1, c.at(c.L.tw_m), c.px);
  a.in_stride = 0;
  a.pre = kPreMulH;
  a.H = c.Ht(0);
  a.H_stride = c.px;
  CTV_TRY(launch_fft_lines(a, c.m, c.n, 1, c.D, c.s), "ifft (columns)");
  FftArgs r = line_args(t1, t2, c.at(c.L.tw_n), c.px);
  r.post = kPostResidual;
  r.scale = 1.0f / (float)((double)c.m * c.n);
  r.sy = c.sy(0);
  r.sy_stride = c.px;
  r.partial = part;
  CTV_TRY(launch_fft_second(r, c.n, c.m, 1, c.D, t2, c.s), "ifft (rows, residual)");
  CTV_TRY(launch_sum_d(part, c.D * residual_blocks(c.m, c.n), 1, 1, out, c.s), "loss");
  return CTV_OK;
}

// F(x) (Eq. 24 summed over d) into *out (device float): data_term with the
// loss trace's float reduction.
ctv_status data_term_f(const Ctx& c, const float2* x, float* out) {
  double* part = reinterpret_cast<double*>(c.ws + c.L.part);
  ctv_status st = fft2_to_t(c, x, c.at(c.L.xh), epilogue(kPostStore, 1.0f));
  if (st) return st;
  FftArgs a = line_args(c.at(c.L.xh), c.at(c.L.t1), c.at(c.L.tw_m), c.px);
  a.in_stride = 0;
  a.pre = kPreMulH;
  a.H = c.Ht(0);
  a.H_stride = c.px;
  CTV_TRY(launch_fft_lines(a, c.m, c.n, 1, c.D, c.s), "ifft (columns)");
  FftArgs r = line_args(c.at(c.L.t1), c.at(c.L.t2), c.at(c.L.tw_n), c.px);
  r.post = kPostResidual;
  r.scale = 1.0f / (float)((double)c.m * c.n);
  r.sy = c.sy(0);
  r.sy_stride = c.px;
  r.partial = part;
  CTV_TRY(launch_fft_second(r, c.n, c.m, 1, c.D, c.at(c.L.t2), c.s), "ifft (rows, residual)");
  CTV_TRY(launch_loss_final(part, c.D * residual_blocks(c.m, c.n), out, c.s), "loss");
  return CTV_OK;
}

// x <- P_C(A_d^H [sqrt(y_d) A_d x / |A_d x|]): the measured-modulus projection
// of distance d followed by the projection onto C (one step of the iterative
// projection method), four 2-D transforms with the pointwise work in their
// first / last passes.
ctv_status ip_step(const Ctx& c, int d, int constr, const float2* x, float2* out) {
  const float inv = 1.0f / (float)((double)c.m * c.n);
  float2* xh = c.at(c.L.xh);
  float2* u = c.at(c.L.v);
  ctv_status st = fft2_to_t(c, x, xh, epilogue(kPostStore, 1.0f));
  if (st) return st;
  FftArgs rep = epilogue(kPostReplace, inv);
  rep.sy = c.sy(d);
  rep.sy_stride = 0;
  st = ifft2_from_t(c, xh, c.Ht(d), u, rep, kPreMulH);
  if (st) return st;
  st = fft2_to_t(c, u, xh, epilogue(kPostStore, 1.0f));
  if (st) return st;
  FftArgs pc = epilogue(kPostProjC, inv);
  pc.constr = constr;
  return ifft2_from_t(c, xh, c.Ht(d), out, pc, kPreMulConjH);
}

Ctx make_ctx(const pr_params* p, int m, int n, void* ws, ctv_stream_t stream) {
  return Ctx{m, n, p->num_meas, (long long)m * n, static_cast<char*>(ws), pr_layout(p->num_meas, m, n),
             reinterpret_cast<hipStream_t>(stream)};
}

}  // namespace

extern "C" {

ctv_status ctv_fft2_workspace_size(int32_t batch, int32_t m, int32_t n, size_t* ws_bytes) {
  if (batch < 1) return fail(CTV_ERR_INVALID_ARG, "batch must be >= 1");
  if (!fft_size_ok(m) || !fft_size_ok(n)) return fail(CTV_ERR_UNSUPPORTED, "m and n must be powers of two in [2, 4096]");
  if (!ws_bytes) return fail(CTV_ERR_INVALID_ARG, "ws_bytes is NULL");
  *ws_bytes = align_up((size_t)n * 8) + align_up((size_t)m * 8) + align_up((size_t)batch * m * n * 8);
  return CTV_OK;
}

ctv_status ctv_fft2(int32_t batch, int32_t m, int32_t n, const float* in, float* out, int32_t inverse, void* ws,
                    size_t ws_bytes, ctv_stream_t stream) {
  size_t need = 0;
  ctv_status st = ctv_fft2_workspace_size(batch, m, n, &need);
  if (st) return st;
  if (!in || !out || !ws) return fail(CTV_ERR_INVALID_ARG, "in, out and ws must be non-NULL");
  if (ws_bytes < need) return fail(CTV_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  float2* twn = reinterpret_cast<float2*>(w);
  float2* twm = reinterpret_cast<float2*>(w + align_up((size_t)n * 8));
  float2* tmp = reinterpret_cast<float2*>(w + align_up((size_t)n * 8) + align_up((size_t)m * 8));
  const float2* x = reinterpret_cast<const float2*>(in);
  float2* y = reinterpret_cast<float2*>(out);
  const long long px = (long long)m * n;
  CTV_TRY(launch_twiddles(twn, n, s), "twiddles");
  CTV_TRY(launch_twiddles(twm, m, s), "twiddles");
  if (!inverse) {
    // rows, transpose, columns (as rows of the transpose), transpose back
    CTV_TRY(launch_fft_lines(line_args(x, y, twn, px), n, m, -1, batch, s), "fft (rows)");
    CTV_TRY(launch_transpose(y, tmp, m, n, batch, s), "transpose");
    CTV_TRY(launch_fft_lines(line_args(tmp, tmp, twm, px), m, n, -1, batch, s), "fft (columns)");
    CTV_TRY(launch_transpose(tmp, y, n, m, batch, s), "transpose");
  } else {
    CTV_TRY(launch_transpose(x, tmp, m, n, batch, s), "transpose");
    CTV_TRY(launch_fft_lines(line_args(tmp, tmp, twm, px), m, n, 1, batch, s), "ifft (columns)");
    CTV_TRY(launch_transpose(tmp, y, n, m, batch, s), "transpose");
    FftArgs a = line_args(y, y, twn, px);
    a.scale = (float)(1.0 / ((double)m * n));
    CTV_TRY(launch_fft_lines(a, n, m, 1, batch, s), "ifft (rows)");
  }
  return CTV_OK;
}

ctv_status pr_workspace_size(const pr_params* p, int32_t m, int32_t n, size_t* ws_bytes) {
  ctv_status st = validate_pr(p, m, n, false);
  if (st) return st;
  if (!ws_bytes) return fail(CTV_ERR_INVALID_ARG, "ws_bytes is NULL");
  *ws_bytes = pr_layout(p->num_meas, m, n).total;
  return CTV_OK;
}

ctv_status pr_forward(const pr_params* p, int32_t m, int32_t n, const float* x, float* out, void* ws,
                      size_t ws_bytes, ctv_stream_t stream) {
  ctv_status st = validate_pr(p, m, n, false);
  if (st) return st;
  if (!x || !out || !ws) return fail(CTV_ERR_INVALID_ARG, "x, out and ws must be non-NULL");
  Ctx c = make_ctx(p, m, n, ws, stream);
  if (ws_bytes < c.L.total) return fail(CTV_ERR_WORKSPACE, "workspace too small");
  st = build_tables(c, p, nullptr);
  if (st) return st;
  st = fft2_to_t(c, reinterpret_cast<const float2*>(x), c.at(c.L.xh), epilogue(kPostStore, 1.0f));
  if (st) return st;
  float2* o = reinterpret_cast<float2*>(out);
  FftArgs a = line_args(c.at(c.L.xh), c.at(c.L.t1), c.at(c.L.tw_m), c.px);
  a.in_stride = 0;
  a.pre = kPreMulH;
  a.H = c.Ht(0);
  a.H_stride = c.px;
  CTV_TRY(launch_fft_lines(a, m, n, 1, c.D, c.s), "ifft (columns)");
  FftArgs b = line_args(c.at(c.L.t1), o, c.at(c.L.tw_n), c.px);
  b.scale = 1.0f / (float)((double)m * n);
  CTV_TRY(launch_fft_second(b, n, m, 1, c.D, o, c.s), "ifft (rows)");
  return CTV_OK;
}

ctv_status pr_gradient(const pr_params* p, int32_t m, int32_t n, const float* y, const float* x, float* grad,
                       float* loss, void* ws, size_t ws_bytes, ctv_stream_t stream) {
  ctv_status st = validate_pr(p, m, n, false);
  if (st) return st;
  if (!y || !x || !grad || !ws) return fail(CTV_ERR_INVALID_ARG, "y, x, grad and ws must be non-NULL");
  Ctx c = make_ctx(p, m, n, ws, stream);
  if (ws_bytes < c.L.total) return fail(CTV_ERR_WORKSPACE, "workspace too small");
  st = build_tables(c, p, y);
  if (st) return st;
  return gradient(c, reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(grad), false, 0.0f, loss);
}

ctv_status pr_prox_grad(const pr_params* p, int32_t m, int32_t n, const float* y, float* x, float* loss_trace,
                        float* gamma_trace, void* ws, size_t ws_bytes, ctv_stream_t stream) {
  ctv_status st = validate_pr(p, m, n, true);
  if (st) return st;
  if (!y || !x || !ws) return fail(CTV_ERR_INVALID_ARG, "y, x and ws must be non-NULL");
  Ctx c = make_ctx(p, m, n, ws, stream);
  if (ws_bytes < c.L.total) return fail(CTV_ERR_WORKSPACE, "workspace too small");
  st = build_tables(c, p, y);
  if (st) return st;
  float2* xcur = c.at(c.L.xcur);
  float2* xprev = c.at(c.L.xprev);
  float2* z = c.at(c.L.z);
  float2* v = c.at(c.L.v);
  float2* g = c.at(c.L.g);
  float2* acc = c.at(c.L.acc);
  float2* syc = c.at(c.L.syc);
  double* lsv = reinterpret_cast<double*>(c.ws + c.L.lsv);
  double* lsp = reinterpret_cast<double*>(c.ws + c.L.lsp);
  const float inv = 1.0f / (float)((double)m * n);
  if (p->init_backprop) {
    // x0 = (1/D) sum_d A_d^H sqrt(y_d): the directly back-propagated field (Section VI-A)
    CTV_TRY(launch_sqrt_y(y, c.atf(c.L.sy), syc, (long long)c.D * c.px, c.s), "sqrt(y)");
    st = accumulate_spectra(c, syc, acc);
    if (st) return st;
    st = ifft2_from_t(c, acc, nullptr, xcur, epilogue(kPostStore, inv / (float)c.D));
    if (st) return st;
  } else {
    CTV_TRY(launch_copy_c(reinterpret_cast<const float2*>(x), xcur, c.px, c.s), "copy");
  }
  // x_{-1} = x_0 (the first momentum weight is 0, and x_0 - x_{-1} must be finite)
  CTV_TRY(launch_copy_c(xcur, xprev, c.px, c.s), "copy");
  float gamma = p->gamma > 0.0f ? p->gamma : 1.0f / (float)c.D;
  Tiling tl;
  st = choose_tiling(&p->inner, m, n, 1, &tl, p->inner.schedule != CTV_S_FLOW);
  if (st) return st;
  const int Kin = p->inner.iters;
  std::vector<float> beta;
  momentum_table(p->inner.method, Kin + 1, beta);
  float* fws = reinterpret_cast<float*>(c.ws + c.L.fgp);
  const size_t st_floats = state_bytes(1, m, n) / 4;
  float* fA = fws;
  float* fB = fws + ((st_floats + 63) & ~(size_t)63);
  // warm start (K_in > 0 only; a prox of zero iterations is P_C(v) either way)
  const bool warm = p->warm_start && Kin > 0;
  float* wcur = reinterpret_cast<float*>(c.ws + c.L.warm);
  float* wnext = wcur + align_up(state_bytes(1, m, n)) / 4;
  bool have_warm = false;

  // x_k = prox_{gamma R}(v) into xnew: Algorithm 2 with lambda = tau gamma from
  // q_0 = 0 or the warm dual; with the warm start the last launch also stores
  // its state.
  float2* xnew = xprev;
  auto prox = [&](float lam) -> ctv_status {
    // A weight the denoiser rejects (0 < tau gamma < 1e-12, reachable only by
    // backtracking far) is taken as 0: P_C alone, within 6 tau gamma per pixel.
    if (lam < kMinLambda) lam = 0.0f;
    int kk = 0;
    const float* src = (warm && have_warm) ? wcur : nullptr;
    do {
      const int Tl = even_split(tl.T, Kin - kk);
      const bool last = (kk + Tl == Kin);
      float* dst = last ? (warm ? wnext : nullptr) : (src == fA ? fB : fA);
      ctv_status e = fgp_launch(&p->inner, tl, 1, m, n, reinterpret_cast<const float*>(v), nullptr, &lam, beta, kk,
                                Tl, src, dst, last ? reinterpret_cast<float*>(xnew) : nullptr, c.s);
      if (e) return e;
      src = dst;
      kk += Tl;
    } while (kk < Kin);
    return CTV_OK;
  };

  // xcur / xprev hold the two latest iterates; z_k = x_{k-1} + b_k (x_{k-1} - x_{k-2})
  // (Algorithm 1, lines 4-5) is formed in the first pass of the gradient's
  // transform, and the prox writes x_k over x_{k-2}.
  double t = 1.0;
  float b = 0.0f;  // z_1 = x_0
  for (int k = 0; k < p->outer_iters; ++k) {
    const Extrapolate ex{xprev, b, z};
    xnew = xprev;
    if (!p->line_search) {
      // v = z_k - gamma grad F(z_k)  (Algorithm 1, line 3's argument)
      st = gradient(c, xcur, v, true, gamma, loss_trace ? loss_trace + k : nullptr, &ex);
      if (st) return st;
      st = prox((float)((double)p->tau * gamma));
      if (st) return st;
    } else {
      st = gradient(c, xcur, g, false, 0.0f, loss_trace ? loss_trace + k : nullptr, &ex);
      if (st) return st;
      CTV_TRY(launch_sum_d(reinterpret_cast<const double*>(c.ws + c.L.part), c.D * residual_blocks(m, n), 1, 1,
                           lsv, c.s), "loss");
      for (int trial = 0;; ++trial) {
        CTV_TRY(launch_grad_step(z, g, gamma, v, c.px, c.s), "gradient step");
        st = prox((float)((double)p->tau * gamma));
        if (st) return st;
        if (trial == p->ls_max_trials - 1) break;
        st = data_term(c, xnew, lsv + 1);
        if (st) return st;
        CTV_TRY(launch_ls_dots(g, xnew, z, c.px, lsp, c.s), "line search");
        CTV_TRY(launch_sum_d(lsp, kLsBlocks, 2, 2, lsv + 2, c.s), "line search");
        double h[4];
        CTV_TRY(hipMemcpyAsync(h, lsv, sizeof(h), hipMemcpyDeviceToHost, c.s), "line search readback");
        CTV_TRY(hipStreamSynchronize(c.s), "line search readback");
        if (h[1] <= h[0] + h[2] + h[3] / (2.0 * (double)gamma)) break;
        gamma *= p->ls_shrink;
      }
    }
    if (gamma_trace) CTV_TRY(launch_fill_f32(gamma_trace + k, gamma, 1, c.s), "gamma trace");
    if (warm) {
      // next prox starts at (q, r) = (q_K, q_K) of this one
      std::swap(wcur, wnext);
      CTV_TRY(launch_copy_c(reinterpret_cast<const float2*>(wcur), reinterpret_cast<float2*>(wcur) + 2 * c.px,
                            2 * c.px, c.s), "warm start");
      have_warm = true;
    }
    // t_{k+1} and the weight (t_k - 1)/t_{k+1} of z_{k+1} = x_k + b (x_k - x_{k-1})
    // (lines 4-5; z_{k+1} is formed by the next gradient)
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    b = p->accelerate ? (float)((t - 1.0) / tn) : 0.0f;
    std::swap(xcur, xprev);
    t = tn;
  }
  CTV_TRY(launch_copy_c(xcur, reinterpret_cast<float2*>(x), c.px, c.s), "copy");
  return CTV_OK;
}

ctv_status pr_ip(const pr_params* p, int32_t m, int32_t n, const float* y, float* x, float* loss_trace, void* ws,
                 size_t ws_bytes, ctv_stream_t stream) {
  ctv_status st = validate_pr(p, m, n, false);
  if (st) return st;
  st = validate_params(&p->inner);
  if (st) return st;
  if (p->outer_iters < 0) return fail(CTV_ERR_INVALID_ARG, "outer_iters must be >= 0");
  if (!y || !x || !ws) return fail(CTV_ERR_INVALID_ARG, "y, x and ws must be non-NULL");
  Ctx c = make_ctx(p, m, n, ws, stream);
  if (ws_bytes < c.L.total) return fail(CTV_ERR_WORKSPACE, "workspace too small");
  st = build_tables(c, p, y);
  if (st) return st;
  float2* xcur = c.at(c.L.xcur);
  if (p->init_backprop) {
    float2* syc = c.at(c.L.syc);
    float2* acc = c.at(c.L.acc);
    CTV_TRY(launch_sqrt_y(y, c.atf(c.L.sy), syc, (long long)c.D * c.px, c.s), "sqrt(y)");
    st = accumulate_spectra(c, syc, acc);
    if (st) return st;
    st = ifft2_from_t(c, acc, nullptr, xcur, epilogue(kPostStore, 1.0f / (float)((double)m * n) / (float)c.D));
    if (st) return st;
  } else {
    CTV_TRY(launch_copy_c(reinterpret_cast<const float2*>(x), xcur, c.px, c.s), "copy");
  }
  for (int k = 0; k < p->outer_iters; ++k) {
    if (loss_trace) {
      st = data_term_f(c, xcur, loss_trace + k);
      if (st) return st;
    }
    for (int d = 0; d < c.D; ++d) {
      st = ip_step(c, d, p->inner.constraint, xcur, xcur);
      if (st) return st;
    }
  }
  CTV_TRY(launch_copy_c(xcur, reinterpret_cast<float2*>(x), c.px, c.s), "copy");
  return CTV_OK;
}

}  // extern "C"
