// Host side of the C ABI: argument validation, workspace layout, the FP64
// momentum schedule of Algorithm 2, and the launch schedule of the fused
// forward kernel (plain batches). Batched plans, the adjoint and the
// phase-retrieval driver live in their own translation units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctv.h"
#include "ctv_host.hpp"
#include "ctv_kernels.hpp"

namespace ctv {

thread_local std::string g_last_error;

// Test hook of the dataflow schedule (ctv_debug_flow_fail_waits).
static std::atomic<int> g_flow_fail_waits{0};

ctv_status fail(ctv_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ctv_status hip_fail(hipError_t e, const char* where) {
  return fail(CTV_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

ctv_status validate_params(const ctv_params* p) {
  if (!p) return fail(CTV_ERR_INVALID_ARG, "params is NULL");
  if (p->struct_size != sizeof(ctv_params)) return fail(CTV_ERR_INVALID_ARG, "ctv_params.struct_size mismatch");
  if (p->tv_kind < CTV_TV_1I || p->tv_kind > CTV_TV_2A) return fail(CTV_ERR_INVALID_ARG, "unknown tv_kind");
  if (p->constraint != CTV_C_NONE && p->constraint != CTV_C_MODULUS)
    return fail(CTV_ERR_INVALID_ARG, "unknown constraint");
  if (!(p->alpha >= 0.0f && p->alpha <= 1.0f)) return fail(CTV_ERR_INVALID_ARG, "alpha must lie in [0, 1]");
  if (p->iters < 0) return fail(CTV_ERR_INVALID_ARG, "iters must be >= 0");
  if (p->fuse < 0 || p->fuse > kMaxFuse) return fail(CTV_ERR_INVALID_ARG, "fuse must lie in [0, 16]");
  if (p->method != CTV_M_FGP && p->method != CTV_M_GP) return fail(CTV_ERR_INVALID_ARG, "unknown method");
  if (p->schedule < CTV_S_AUTO || p->schedule > CTV_S_FLOW) return fail(CTV_ERR_INVALID_ARG, "unknown schedule");
  return CTV_OK;
}

ctv_status validate_lambda(float lam) {
  if (!(lam >= 0.0f) || !std::isfinite(lam)) return fail(CTV_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  // The dual step 1/(8 lambda), the squared dual norms it feeds and the
  // backward's 1/(8 lambda^2) must stay finite in float32: below ~2e-20 the
  // latter overflows, and for subnormal lambda the step itself is infinite.
  if (lam > 0.0f && lam < kMinLambda)
    return fail(CTV_ERR_INVALID_ARG, "lambda must be 0 or >= 1e-12 (smaller values overflow the float32 dual step)");
  return CTV_OK;
}

Radii make_radii(int kind, float alpha) {
  Radii R;
  if (kind == CTV_TV_2I || kind == CTV_TV_2A) {
    const double a = alpha, s = 1.0 - (double)alpha;
    R.ra = (float)a;
    R.ra2 = (float)(a * a);
    R.sa = (float)s;
    R.sa2 = (float)(s * s);
  } else {
    R.ra = R.ra2 = R.sa = R.sa2 = 1.0f;
  }
  return R;
}

void momentum_table(int method, int kmax, std::vector<float>& beta) {
  // beta[k] = (t_k - 1) / t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
  // (Algorithm 2, lines 4-5), evaluated in float64 and rounded once. The plain
  // gradient projection (Eq. 21) keeps every beta at 0: r_k = q_{k-1} exactly.
  beta.assign((size_t)kmax + 2, 0.0f);
  if (method == CTV_M_GP) return;
  double t = 1.0;
  for (int k = 1; k <= kmax + 1; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    beta[(size_t)k] = (float)((t - 1.0) / tn);
    t = tn;
  }
}

float step_of(float lam) {
  // 1/(16 lambda^2) times the 2 lambda of Eq. (19); lambda = 0 gives a zero
  // step, which keeps q = 0 and returns x = P_C(b) exactly.
  return lam > 0.0f ? (float)(1.0 / (8.0 * (double)lam)) : 0.0f;
}

bool valid_tile_shape(const TileShape& ts) {
  if (ts.sweep()) return ts.rows_per_thread >= 16 && ts.rows_per_thread <= 1024 && ts.rows_per_thread % 4 == 0;
  if (ts.waves > 0)
    return (ts.waves == 4 && ts.rows_per_thread == 8) ||
           ((ts.waves == 8 || ts.waves == 16) && (ts.rows_per_thread == 4 || ts.rows_per_thread == 8)) ||
           (ts.waves == 12 && ts.rows_per_thread == 4);
  return ts.rows_per_thread == 4 || ts.rows_per_thread == 8 || ts.rows_per_thread == 16;
}

void clamp_fuse(Tiling* t, int iters) {
  // halo H <= (min(64, rows) - 1) / 2 keeps at least one output row and column;
  // the epilogue launch needs H = T + 1.
  const int hmax = (std::min(64, t->shape.rows()) - 1) / 2;
  t->T = std::min(t->T, hmax - 1);
  if (t->shape.sweep()) t->T = std::min(t->T, kSweepMaxFuse);
  if (iters > 0) t->T = std::min(t->T, iters);
  t->T = std::max(t->T, 1);
}

ctv_status choose_tiling(const ctv_params* p, int m, int n, int batch, Tiling* out, bool use_tuned) {
  Tiling t;
  t.shape.waves = 8;
  t.shape.rows_per_thread = 8;
  // Default from the tiling sweep on MI355X (2048^2, K = 200): 8 waves x 8 rows
  // (64 x 64 regions) with 8 fused iterations.
  t.T = 8;
  if (p->tile_waves != 0 || p->tile_rows != 0) {
    if (p->tile_waves == 0 || p->tile_rows == 0) return fail(CTV_ERR_INVALID_ARG, "tile_waves and tile_rows must be set together");
    t.shape.waves = p->tile_waves == -1 ? 0 : p->tile_waves;   // -1: LDS tile; kSweepShape: row sweep
    t.shape.rows_per_thread = p->tile_rows;
    if (p->tile_waves < kSweepShape || !valid_tile_shape(t.shape))
      return fail(CTV_ERR_INVALID_ARG, "unsupported tile shape");
  } else if (use_tuned && p->fuse == 0) {
    Tiling tuned;
    if (tuned_lookup(plain_tune_key(p, batch, m, n), &tuned) && valid_tile_shape(tuned.shape)) t = tuned;
  }
  if (p->fuse > 0) t.T = p->fuse;
  clamp_fuse(&t, p->iters);
  *out = t;
  return CTV_OK;
}

size_t state_bytes(long long batch, long long m, long long n) { return (size_t)(batch * 2 * m * n * 16); }

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

int gap_blocks_per_image(long long px) {
  long long b = (px + 1023) / 1024;
  return (int)std::max(1LL, std::min(256LL, b));
}

// Largest halo of the 8 x 8 tile (fuse <= 16): bounds the flow bookkeeping.
static int flow_max_halo() { return kMaxFuse; }

// Live-tile lists: tilings whose output tiles are at least 16 x 16 pixels have
// at most live_cap tiles; each of kLiveSlots tilings keeps flags[cap] and
// live[1 + cap].
constexpr int kLiveSlots = 3;
static long long live_cap(int m, int n) { return (long long)((m + 15) / 16) * ((n + 15) / 16); }
static size_t live_ints(int m, int n) { return (size_t)kLiveSlots * (2 * live_cap(m, n) + 1); }

size_t denoise_ws_bytes(int batch, int m, int n) {
  const size_t st = align_up(state_bytes(batch, m, n));
  const size_t gap = align_up((size_t)batch * gap_blocks_per_image((long long)m * n) * sizeof(double));
  const size_t flow = align_up((size_t)flow_ints(std::min(batch, kPlainChunk), m, n, flow_max_halo()) * 4);
  return 2 * st + gap + flow + align_up(live_ints(m, n) * 4);
}

ctv_status fgp_launch(const ctv_params* p, const Tiling& tl, int cb, int m, int n, const float* b,
                      const uint8_t* support, const float* lam, const std::vector<float>& beta, int k, int Tl,
                      const float* src, float* dst, float* x, hipStream_t s, float* r_hist,
                      long long r_hist_stride, const int* live) {
  if (r_hist && (tl.shape.waves != 8 || tl.shape.rows_per_thread != 8))
    return fail(CTV_ERR_INVALID_ARG, "r history needs the 8 x 8 column tile");
  FgpPlainArgs a;
  std::memset(&a, 0, sizeof(a));
  a.b = b;
  a.mask = support;
  a.m = m;
  a.n = n;
  a.R = make_radii(p->tv_kind, p->alpha);
  for (int i = 0; i < cb; ++i) {
    a.lam[i] = lam[i];
    a.c[i] = step_of(lam[i]);
  }
  a.st_in = src;
  a.st_out = dst;
  a.x = x;
  a.r_hist = r_hist;
  a.r_hist_stride = r_hist_stride;
  if (live && ((tl.shape.waves <= 0 && !tl.shape.sweep()) || r_hist))
    return fail(CTV_ERR_INVALID_ARG, "internal: live-tile lists need the column or row-sweep tiles");
  a.live = live;
  a.T = Tl;
  a.halo = std::max(1, Tl + (x ? 1 : 0));
  for (int i = 0; i < kMaxFuse; ++i) a.beta[i] = (i < Tl) ? beta[(size_t)(k + 1 + i)] : 0.0f;
  const int oh = tl.shape.out_rows(a.halo);
  a.tiles_x = (n + (64 - 2 * a.halo) - 1) / (64 - 2 * a.halo);
  a.tiles_y = (m + oh - 1) / oh;
  a.sweep_rows = tl.shape.sweep() ? tl.shape.rows_per_thread : 0;
  hipError_t e = launch_fgp_plain(a, p->tv_kind, p->constraint, tl.shape, cb, s);
  if (e != hipSuccess) return hip_fail(e, "fgp launch");
  return CTV_OK;
}

}  // namespace ctv

using namespace ctv;

extern "C" {

int32_t ctv_version(void) { return 100; }

const char* ctv_last_error(void) { return g_last_error.c_str(); }

ctv_status ctv_debug_flow_fail_waits(int32_t on) {
  g_flow_fail_waits.store(on ? 1 : 0);
  return CTV_OK;
}

ctv_status ctv_workspace_size(const ctv_params* p, int32_t batch, int32_t m, int32_t n,
                              int32_t ckpt_every, size_t* ws_bytes, size_t* saved_bytes) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (batch < 1 || m < 1 || n < 1) return fail(CTV_ERR_INVALID_ARG, "batch, m and n must be >= 1");
  if (ckpt_every < 0) return fail(CTV_ERR_INVALID_ARG, "ckpt_every must be >= 0");
  if (ws_bytes) *ws_bytes = denoise_ws_bytes(batch, m, n);
  if (saved_bytes) {
    long long slots = 0;
    if (ckpt_every > 0 && p->iters > 0) slots = (p->iters + ckpt_every - 1) / ckpt_every - 1;
    *saved_bytes = (size_t)slots * state_bytes(batch, m, n);
  }
  return CTV_OK;
}

ctv_status ctv_tiling(const ctv_params* p, int32_t batch, int32_t m, int32_t n, int32_t* fuse_out,
                      int32_t* region_rows_out, int32_t* tile_waves_out, int32_t* tile_rows_out) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (batch < 1 || m < 1 || n < 1) return fail(CTV_ERR_INVALID_ARG, "batch, m and n must be >= 1");
  Tiling t;
  st = choose_tiling(p, m, n, batch, &t, p->schedule != CTV_S_FLOW);
  if (st) return st;
  if (fuse_out) *fuse_out = t.T;
  if (region_rows_out) *region_rows_out = t.shape.rows();
  if (tile_waves_out) *tile_waves_out = (t.shape.waves > 0 || t.shape.sweep()) ? t.shape.waves : -1;
  if (tile_rows_out) *tile_rows_out = t.shape.rows_per_thread;
  return CTV_OK;
}

ctv_status ctv_denoise(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                       const float* lambda_host, const uint8_t* support, float* x, double* gap,
                       const float* state_in, int32_t k0, float* state_out, int32_t ckpt_every,
                       float* saved, void* ws, size_t ws_bytes, ctv_stream_t stream) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (batch < 1 || m < 1 || n < 1) return fail(CTV_ERR_INVALID_ARG, "batch, m and n must be >= 1");
  if (!b || !x || !lambda_host) return fail(CTV_ERR_INVALID_ARG, "b, x and lambda_host must be non-NULL");
  if (b == x) return fail(CTV_ERR_INVALID_ARG, "x must not alias b");
  if (state_out && state_out == state_in) return fail(CTV_ERR_INVALID_ARG, "state_out must not alias state_in");
  for (int i = 0; i < batch; ++i) {
    st = validate_lambda(lambda_host[i]);
    if (st) return st;
  }
  if (k0 < 0) return fail(CTV_ERR_INVALID_ARG, "k0 must be >= 0");
  if (!state_in && k0 != 0) return fail(CTV_ERR_INVALID_ARG, "k0 > 0 requires state_in");
  if (ckpt_every < 0) return fail(CTV_ERR_INVALID_ARG, "ckpt_every must be >= 0");
  if (ckpt_every > 0 && state_in) return fail(CTV_ERR_INVALID_ARG, "checkpoints require a cold start");
  const long long slots = (ckpt_every > 0 && p->iters > 0) ? (p->iters + ckpt_every - 1) / ckpt_every - 1 : 0;
  if (slots > 0 && !saved) return fail(CTV_ERR_INVALID_ARG, "saved is NULL but checkpoints are requested");
  if ((long long)k0 + p->iters > (1LL << 30)) return fail(CTV_ERR_INVALID_ARG, "k0 + iters too large");
  if (!ws) return fail(CTV_ERR_INVALID_ARG, "ws is NULL");
  const size_t need = denoise_ws_bytes(batch, m, n);
  if (ws_bytes < need) return fail(CTV_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long px = (long long)m * n;
  const size_t st_full = state_bytes(batch, m, n);
  char* wsb = static_cast<char*>(ws);
  float* bufA = reinterpret_cast<float*>(wsb);
  float* bufB = reinterpret_cast<float*>(wsb + align_up(st_full));
  double* partial = reinterpret_cast<double*>(wsb + 2 * align_up(st_full));
  int* flow_mem = reinterpret_cast<int*>(
      wsb + 2 * align_up(st_full) + align_up((size_t)batch * gap_blocks_per_image(px) * sizeof(double)));
  int* live_mem = reinterpret_cast<int*>(
      reinterpret_cast<char*>(flow_mem) +
      align_up((size_t)flow_ints(std::min(batch, kPlainChunk), m, n, flow_max_halo()) * 4));
  Tiling tl;
  st = choose_tiling(p, m, n, batch, &tl, p->schedule != CTV_S_FLOW);
  if (st) return st;
  const bool flow_ok = ckpt_every == 0 && p->iters > 0 && tl.shape.waves == 8 && tl.shape.rows_per_thread == 8;
  if (p->schedule == CTV_S_FLOW && !flow_ok)
    return fail(CTV_ERR_INVALID_ARG, "the dataflow schedule needs ckpt_every = 0, iters > 0 and the 8 x 8 tile");
  // Automatic choice: one launch per fused step. The dataflow launch moves the
  // dual state through device-coherent accesses, which on MI355X cost more
  // (2048^2, K = 200: 279 vs 346 G px-it/s) than the launch tail it removes.
  const bool use_flow = flow_ok && p->schedule == CTV_S_FLOW;
  // an image that fits in one 8 x 8 column tile runs without a halo, all
  // iterations of a chunk in one launch (same results as per-step launches)
  const bool use_single = !use_flow && p->schedule == CTV_S_AUTO && ckpt_every == 0 && m <= 64 && n <= 64 &&
                          tl.shape.waves == 8 && tl.shape.rows_per_thread == 8;
  std::vector<float> beta;
  momentum_table(p->method, k0 + p->iters + 1, beta);
  const Radii R = make_radii(p->tv_kind, p->alpha);

  for (int c0 = 0; c0 < batch; c0 += kPlainChunk) {
    const int cb = std::min(kPlainChunk, batch - c0);
    const long long img_px = px * c0;            // pixel offset of the chunk
    const long long st_off = 2 * px * c0 * 4;    // float offset of the chunk in a state buffer
    const float* src = state_in ? state_in + st_off : nullptr;
    int k = k0;
    const int kend = k0 + p->iters;
    if (use_single) {
      do {
        const int Kc = std::min(kFlowMaxIters, kend - k);
        const bool last = (k + Kc == kend);
        FgpSingleArgs sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.b = b + 2 * img_px;
        sa.mask = support;
        sa.st_in = src;
        float* other = (src == bufA + st_off) ? bufB + st_off : bufA + st_off;
        sa.st_out = last ? (state_out ? state_out + st_off : (gap ? other : nullptr)) : other;
        sa.x = last ? x + 2 * img_px : nullptr;
        sa.m = m;
        sa.n = n;
        sa.T = Kc;
        sa.R = R;
        for (int i = 0; i < cb; ++i) {
          sa.lam[i] = lambda_host[c0 + i];
          sa.c[i] = step_of(lambda_host[c0 + i]);
        }
        for (int i = 0; i < Kc; ++i) sa.beta[i] = beta[(size_t)(k + 1 + i)];
        hipError_t e = launch_fgp_single(sa, p->tv_kind, p->constraint, cb, s);
        if (e != hipSuccess) return hip_fail(e, "fgp single-tile launch");
        src = sa.st_out;
        k += Kc;
      } while (k < kend);
    } else if (use_flow) {
      // chunks of whole fused steps, each one persistent launch
      const int chunk_iters = (kFlowMaxIters / tl.T) * tl.T;
      while (k < kend) {
        const int Kc = std::min(chunk_iters, kend - k);
        const bool final_chunk = (k + Kc == kend);
        FgpFlowArgs fa;
        std::memset(&fa, 0, sizeof(fa));
        fa.b = b + 2 * img_px;
        fa.mask = support;
        fa.st_in = src;
        // buf0 holds this chunk's input when it comes from the workspace
        float* in_ws = (src == bufB + st_off) ? bufB + st_off : bufA + st_off;
        fa.buf0 = in_ws;
        fa.buf1 = (in_ws == bufA + st_off) ? bufB + st_off : bufA + st_off;
        fa.m = m;
        fa.n = n;
        fa.batch = cb;
        fa.halo = tl.T;
        fa.T = tl.T;
        fa.steps = (Kc + tl.T - 1) / tl.T;
        fa.T_last = Kc - (fa.steps - 1) * tl.T;
        fa.tiles_x = (n + (64 - 2 * fa.halo) - 1) / (64 - 2 * fa.halo);
        fa.tiles_y = (m + (tl.shape.rows() - 2 * fa.halo) - 1) / (tl.shape.rows() - 2 * fa.halo);
        float* last_state = (fa.steps % 2 == 0) ? fa.buf0 : fa.buf1;  // written by the last compute step
        fa.st_out = (final_chunk && state_out) ? state_out + st_off : nullptr;
        fa.x = final_chunk ? x + 2 * img_px : nullptr;
        fa.R = R;
        for (int i = 0; i < cb; ++i) {
          fa.lam[i] = lambda_host[c0 + i];
          fa.c[i] = step_of(lambda_host[c0 + i]);
        }
        for (int i = 0; i < Kc; ++i) fa.beta[i] = beta[(size_t)(k + 1 + i)];
        const long long ints = flow_ints(cb, m, n, fa.halo);
        fa.counter = flow_mem;
        fa.err = flow_mem + 1;
        fa.preset_err = g_flow_fail_waits.load();
        fa.done = flow_mem + 64;
        hipError_t e = launch_zero_f4(reinterpret_cast<float*>(flow_mem), (ints + 3) / 4, s);
        if (e == hipSuccess) e = launch_fgp_flow(fa, p->tv_kind, p->constraint, s);
        if (e != hipSuccess) return hip_fail(e, "fgp flow launch");
        src = fa.st_out ? fa.st_out : last_state;
        k += Kc;
      }
    } else {
      // With a support and a cold start, the dual stays zero at pixels that
      // neither lie in the support nor have a support pixel below or to the
      // right of them (x = 0 there too). Launches that read and write only the
      // workspace buffers run just the tiles holding other pixels, from a
      // live-tile list built once per tiling: the first list also stores the
      // zeros at those pixels of both buffers, the one of the launch that
      // writes x stores x = 0 in its skipped tiles. Launches into checkpoint
      // slots or a caller's state buffer run every tile. Results are bitwise
      // those of running every tile.
      const bool may_skip = support && !state_in && (tl.shape.waves > 0 || tl.shape.sweep());
      int slot_h[kLiveSlots], slot_x[kLiveSlots], used = 0;
      bool zeroed = false;
      const size_t slot_ints = 2 * live_cap(m, n) + 1;
      do {
        const int seg_end = ckpt_every > 0 ? std::min(kend, (k / ckpt_every + 1) * ckpt_every) : kend;
        const int Tl = even_split(tl.T, seg_end - k);
        const bool last = (k + Tl == kend);
        float* dst;
        float* other = (src == bufA + st_off) ? bufB + st_off : bufA + st_off;
        if (last)
          dst = state_out ? state_out + st_off : (gap ? other : nullptr);
        else if (ckpt_every > 0 && (k + Tl) % ckpt_every == 0)
          dst = saved + (size_t)((k + Tl) / ckpt_every - 1) * (st_full / 4) + st_off;
        else
          dst = other;
        const int* live = nullptr;
        const bool dst_ws = !dst || dst == bufA + st_off || dst == bufB + st_off;
        if (may_skip && dst_ws) {
          const int H = std::max(1, Tl + (last ? 1 : 0));
          const int OW = 64 - 2 * H, OH = tl.shape.out_rows(H);
          const int rows = OH + 2 * H;   // region rows of the scan's tiling
          const long long tiles = (long long)((n + OW - 1) / OW) * ((m + OH - 1) / OH);
          int slot = -1;
          for (int i = 0; i < used; ++i)
            if (slot_h[i] == H && slot_x[i] == (last ? 1 : 0)) slot = i;
          if (slot < 0 && used < kLiveSlots && OW >= 16 && OH >= 16 && tiles <= live_cap(m, n)) {
            slot = used++;
            slot_h[slot] = H;
            slot_x[slot] = last ? 1 : 0;
            LiveScanArgs la;
            la.mask = support;
            la.m = m;
            la.n = n;
            la.halo = H;
            la.rows = rows;
            la.tiles_x = (n + OW - 1) / OW;
            la.tiles_y = (m + OH - 1) / OH;
            la.flags = live_mem + slot * slot_ints;
            la.zero_st = zeroed ? 0 : 1;
            la.st0 = bufA + st_off;
            la.st1 = bufB + st_off;
            la.x = last ? x + 2 * img_px : nullptr;
            la.batch = cb;
            hipError_t e = launch_live_tiles(la, live_mem + slot * slot_ints + live_cap(m, n), s);
            if (e != hipSuccess) return hip_fail(e, "live-tile scan");
            zeroed = true;
          }
          if (slot >= 0) live = live_mem + slot * slot_ints + live_cap(m, n);
        }
        st = fgp_launch(p, tl, cb, m, n, b + 2 * img_px, support, lambda_host + c0, beta, k, Tl, src, dst,
                        last ? x + 2 * img_px : nullptr, s, nullptr, 0, live);
        if (st) return st;
        src = dst;
        k += Tl;
      } while (k < kend);
    }
    if (gap) {
      GapArgs ga;
      for (int i = 0; i < cb; ++i) ga.lam[i] = lambda_host[c0 + i];
      const float* qstate = src;
      if (!qstate) return fail(CTV_ERR_HIP, "internal: no final state for the gap");
      hipError_t e = launch_gap(x + 2 * img_px, qstate, m, n, cb, p->tv_kind, R, ga, partial,
                                gap_blocks_per_image(px), gap + c0, s);
      if (e != hipSuccess) return hip_fail(e, "gap launch");
    }
  }
  return CTV_OK;
}

}  // extern "C"
