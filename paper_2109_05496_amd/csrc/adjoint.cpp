// Host side of ctv_denoise_backward: segment-wise recomputation from the
// forward checkpoints (fused launches that also store every r_k), the
// Eq. (18) output adjoint, one reverse-step launch per iteration, and the
// deterministic lambda-gradient reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "ctv.h"
#include "ctv_adjoint.hpp"
#include "ctv_host.hpp"
#include "ctv_kernels.hpp"

using namespace ctv;

namespace {

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Reverse steps run up to kMaxRev per launch; every launch of a call uses the
// halo of the longest one, so the tile grid (and the lambda-gradient slot of
// each tile) is the same throughout.
int adj_halo(int ckpt) { return std::min(kMaxRev, std::max(ckpt, 1)) + 1; }
int adj_tiles_x(int n, int h) { return (n + (64 - 2 * h) - 1) / (64 - 2 * h); }
int adj_tiles_y(int m, int h) { return (m + (adj_tile_rows() - 2 * h) - 1) / (adj_tile_rows() - 2 * h); }

struct BwdLayout {
  size_t seg, adj, lam, live, total;
};

BwdLayout layout(int batch, int m, int n, int ckpt) {
  BwdLayout L;
  const size_t st = align_up(state_bytes(batch, m, n));
  const int h = adj_halo(ckpt);
  const size_t tiles = (size_t)adj_tiles_x(n, h) * adj_tiles_y(m, h);
  L.seg = (size_t)std::max(ckpt, 1) * st;
  L.adj = 2 * st;
  L.lam = align_up((size_t)batch * tiles * sizeof(double));
  L.live = align_up((2 * tiles + 1) * sizeof(int));  // flags, then the live-tile list
  L.total = L.seg + L.adj + L.lam + L.live;
  return L;
}

}  // namespace

extern "C" {

ctv_status ctv_backward_workspace_size(const ctv_params* p, int32_t batch, int32_t m, int32_t n, int32_t ckpt_every,
                                       size_t* ws_bytes) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (batch < 1 || m < 1 || n < 1) return fail(CTV_ERR_INVALID_ARG, "batch, m and n must be >= 1");
  if (ckpt_every < 1) return fail(CTV_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  if (!ws_bytes) return fail(CTV_ERR_INVALID_ARG, "ws_bytes is NULL");
  *ws_bytes = layout(batch, m, n, std::min(ckpt_every, std::max(p->iters, 1))).total;
  return CTV_OK;
}

ctv_status ctv_denoise_backward(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                                const float* lambda_host, const uint8_t* support, int32_t ckpt_every,
                                const float* saved, const float* grad_x, float* grad_b, float* grad_lambda,
                                void* ws, size_t ws_bytes, ctv_stream_t stream) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (batch < 1 || m < 1 || n < 1) return fail(CTV_ERR_INVALID_ARG, "batch, m and n must be >= 1");
  if (!b || !lambda_host || !grad_x || !grad_b || !grad_lambda)
    return fail(CTV_ERR_INVALID_ARG, "b, lambda_host, grad_x, grad_b and grad_lambda must be non-NULL");
  if (grad_b == b || grad_b == grad_x) return fail(CTV_ERR_INVALID_ARG, "grad_b must not alias b or grad_x");
  for (int i = 0; i < batch; ++i) {
    st = validate_lambda(lambda_host[i]);
    if (st) return st;
  }
  if (ckpt_every < 1) return fail(CTV_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  const int K = p->iters;
  const int c = std::min(ckpt_every, std::max(K, 1));
  const int nseg = K > 0 ? (K + c - 1) / c : 0;
  if (nseg > 1 && !saved) return fail(CTV_ERR_INVALID_ARG, "saved is NULL but the forward stored checkpoints");
  if (!ws) return fail(CTV_ERR_INVALID_ARG, "ws is NULL");
  const BwdLayout L = layout(batch, m, n, c);
  if (ws_bytes < L.total) return fail(CTV_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.total) + " bytes");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long px = (long long)m * n;
  const size_t st_full = state_bytes(batch, m, n);
  const size_t st_stride = align_up(st_full);
  char* wsb = static_cast<char*>(ws);
  float* seg = reinterpret_cast<float*>(wsb);
  float* adjX = reinterpret_cast<float*>(wsb + L.seg);
  float* adjY = reinterpret_cast<float*>(wsb + L.seg + st_stride);
  double* lam_acc = reinterpret_cast<double*>(wsb + L.seg + L.adj);
  int* live_mem = reinterpret_cast<int*>(wsb + L.seg + L.adj + L.lam);

  // x = P_C(b) for every image when K = 0; lambda = 0 images go through the
  // general path (step 0 keeps q = 0) with a zero lambda gradient.
  if (K == 0) {
    hipError_t e = launch_pc_vjp(b, support, grad_x, grad_b, px, batch, p->constraint, s);
    if (e == hipSuccess) e = launch_zero_f32(grad_lambda, batch, s);
    if (e != hipSuccess) return hip_fail(e, "backward (K = 0)");
    return CTV_OK;
  }

  // Recomputation runs the fused column-tile kernel (default shape), storing
  // r after every iteration; results do not depend on the tiling. A segment
  // of up to 12 iterations is recomputed in one launch (16 x 512^2, c = 10:
  // one launch of 9-10 iterations per segment instead of two measured 5 %
  // faster over the whole backward pass).
  Tiling tl;
  ctv_params tp = *p;
  tp.fuse = std::min(c, 12);
  tp.tile_waves = 0;
  tp.tile_rows = 0;
  tp.iters = c;
  st = choose_tiling(&tp, m, n, batch, &tl);
  if (st) return st;
  std::vector<float> beta;
  momentum_table(p->method, K + 1, beta);
  const int halo = adj_halo(c);
  const int tiles_x = adj_tiles_x(n, halo), tiles_per_img = tiles_x * adj_tiles_y(m, halo);

  for (int c0 = 0; c0 < batch; c0 += kPlainChunk) {
    const int cb = std::min(kPlainChunk, batch - c0);
    const long long img_px = px * c0;
    const long long st_off = 2 * px * c0 * 4;
    AdjStepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.b = b + 2 * img_px;
    a.mask = support;
    a.grad_b = grad_b + 2 * img_px;
    a.grad_x = grad_x + 2 * img_px;
    a.lam_acc = lam_acc + (size_t)c0 * tiles_per_img;
    a.m = m;
    a.n = n;
    a.tiles_x = tiles_x;
    a.tiles_per_img = tiles_per_img;
    a.halo = halo;
    a.R = make_radii(p->tv_kind, p->alpha);
    for (int i = 0; i < cb; ++i) {
      const double lam = lambda_host[c0 + i];
      a.lam[i] = (float)lam;
      a.c[i] = step_of((float)lam);
      a.cc[i] = lam > 0.0 ? (float)(1.0 / (8.0 * lam * lam)) : 0.0f;
    }
    float* cur = adjX + st_off;
    float* nxt = adjY + st_off;
    // With a support the adjoint state stays zero wherever the forward dual
    // does (outside the support, no support pixel below or to the right): the
    // reverse steps run only the tiles holding other pixels, after both
    // adjoint buffers got their zeros there. The output step runs every tile.
    const int* live = nullptr;
    if (support) {
      LiveScanArgs la;
      la.mask = support;
      la.m = m;
      la.n = n;
      la.halo = halo;
      la.rows = adj_tile_rows();
      la.tiles_x = tiles_x;
      la.tiles_y = tiles_per_img / tiles_x;
      la.flags = live_mem;
      la.zero_st = 1;
      la.st0 = cur;
      la.st1 = nxt;
      la.x = nullptr;
      la.batch = cb;
      hipError_t e = launch_live_tiles(la, live_mem + tiles_per_img, s);
      if (e != hipSuccess) return hip_fail(e, "adjoint live-tile scan");
      live = live_mem + tiles_per_img;
    }
    auto slot = [&](int j) { return seg + (size_t)j * (st_stride / 4) + st_off; };
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
      const int ks = sgi * c, ke = std::min(ks + c, K);
      const float* ck = (sgi == 0) ? nullptr : saved + (size_t)(sgi - 1) * (st_full / 4) + st_off;
      // recompute iterations ks+1 .. kstop: slot[j] receives r_{ks+j+2} (plane 1) for
      // every j, and the full state after each launch's last iteration
      const int kstop = (sgi == nseg - 1) ? ke : ke - 1;
      const float* prev = ck;
      for (int k = ks; k < kstop;) {
        const int Tl = even_split(tl.T, kstop - k);
        float* last = slot(k + Tl - 1 - ks);
        st = fgp_launch(p, tl, cb, m, n, a.b, support, lambda_host + c0, beta, k, Tl, prev, last, nullptr, s,
                        slot(k - ks), (long long)(st_stride / 4));
        if (st) return st;
        prev = last;
        k += Tl;
      }
      if (sgi == nseg - 1) {
        for (int i = 0; i < kMaxRev; ++i) a.r[i] = nullptr;
        a.r[0] = slot(ke - ks - 1);  // q_K in plane 0
        a.steps = 0;
        a.adj_in = nullptr;
        a.adj_out = cur;
        hipError_t e = launch_adj_output(a, p->constraint, cb, s);
        if (e != hipSuccess) return hip_fail(e, "adjoint output step");
      }
      // reverse steps ke, ke-1, ..., ks+1, up to kMaxRev per launch; r_k is in
      // plane 1 of slot[k - ks - 2], r_{ks+1} in the checkpoint (zero for k = 1)
      for (int khi = ke; khi >= ks + 1;) {
        const int steps = std::min(kMaxRev, khi - ks);
        for (int i = 0; i < kMaxRev; ++i) {
          const int k = khi - i;
          a.r[i] = (i >= steps) ? nullptr : (k == ks + 1) ? ck : slot(k - ks - 2);
          a.beta[i] = (i < steps && k >= 2) ? beta[(size_t)(k - 1)] : 0.0f;
        }
        a.steps = steps;
        a.adj_in = cur;
        a.adj_out = (khi - steps + 1 == 1) ? nullptr : nxt;
        a.live = live;
        hipError_t e = launch_adj_step(a, p->tv_kind, p->constraint, cb, s);
        if (e != hipSuccess) return hip_fail(e, "adjoint step");
        std::swap(cur, nxt);
        khi -= steps;
      }
    }
    hipError_t e = launch_lam_final(a.lam_acc, tiles_per_img, cb, grad_lambda + c0, s);
    if (e != hipSuccess) return hip_fail(e, "lambda gradient reduction");
  }
  return CTV_OK;
}

}  // extern "C"
