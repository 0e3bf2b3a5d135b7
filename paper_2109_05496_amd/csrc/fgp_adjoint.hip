// Reverse-mode kernels of the K-step FGP map (b, lambda) -> x (Algorithm 2 +
// Eq. 18). The paper does not differentiate its solver; these kernels apply
// the chain rule to the iteration as the forward kernels compute it:
//
//   w_k = b - lambda L^T r_k,  y_k = P_C(w_k),  g_k = r_k + c L(y_k)   (c = 1/(8 lambda))
//   q_k = P_S(g_k),            r_{k+1} = q_k + beta_k (q_k - q_{k-1})
//   x   = P_C(b - lambda L^T q_K)
//
// The adjoint state carried from step k+1 to step k is (A, B) = (qbar_k,
// partial qbar_{k-1}); one reverse step computes
//   gbar = J_PS(g_k)^T A,  ybar = c L^T(gbar),  wbar = J_PC(w_k)^T ybar,
//   rbar = gbar - lambda L(wbar),  bbar += wbar,
//   lambdabar += -<gbar, L y_k>/(8 lambda^2) - <wbar, L^T r_k>,
//   A' = B + (1 + beta_{k-1}) rbar,  B' = -beta_{k-1} rbar.
// Non-smooth points: a ball projection has the identity Jacobian when its
// scale is 1 (norm <= radius) and rho (I - v v^T/|v|^2)/|v| otherwise; a zero
// radius has the zero Jacobian. The duals that do not exist (Q1 on the last
// row, Q2 on the last column) are identically zero in the forward pass, so
// their adjoints are zero here.
//
// Tiles: column-register layout as in the forward kernel (lane = column,
// wave = P consecutive rows, DPP for left/right, LDS for wave-boundary rows).
// Up to kMaxRev reverse steps run per launch; the four stencil stages of a step
// read up/left, down/right, up/left, down/right, which widens the dependence of
// (A, B) by one pixel per step, so a launch of s steps needs a halo of s + 1.
#include <hip/hip_runtime.h>

#include "ctv_adjoint.hpp"
#include "ctv_device.hpp"

namespace ctv {

namespace {

constexpr int kRW = 64;

__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Same operations as proj_c, also returning the scale s (1 when inactive).
template <int CONSTR>
__device__ __forceinline__ float2 proj_c_s(float2 w, bool inside, float& s) {
  if (CONSTR == C_MOD) {
    const float n2 = fmaf(w.x, w.x, w.y * w.y);
    s = fminf(1.0f, rsq(n2));
    const float sm = inside ? s : 0.0f;
    return make_float2(fmaf(w.x, sm, 0.0f), fmaf(w.y, sm, 0.0f));
  }
  s = 1.0f;
  return make_float2(inside ? w.x : 0.0f, inside ? w.y : 0.0f);
}

// J_PC(w)^T ybar.
template <int CONSTR>
__device__ __forceinline__ float2 proj_c_vjp(float2 w, float s, bool inside, float2 yb) {
  if (!inside) return make_float2(0.0f, 0.0f);
  if (CONSTR == C_MOD && s < 1.0f) {
    // s (I - w w^T s^2) yb, with s = 1/|w|
    const float d = (w.x * yb.x + w.y * yb.y) * (s * s);
    return make_float2(s * (yb.x - w.x * d), s * (yb.y - w.y * d));
  }
  return yb;
}

// J^T a for the projection of v onto the ball of radius rho with scale f =
// min(1, rho/|v|).
__device__ __forceinline__ void ball_vjp2(float vx, float vy, float ax, float ay, float f, float rho,
                                          float& ox, float& oy) {
  if (rho <= 0.0f) {
    ox = oy = 0.0f;
  } else if (f < 1.0f) {
    const float n2 = vx * vx + vy * vy;
    const float d = (vx * ax + vy * ay) / n2;
    ox = f * (ax - vx * d);
    oy = f * (ay - vy * d);
  } else {
    ox = ax;
    oy = ay;
  }
}

template <int KIND>
__device__ __forceinline__ float4 proj_s_vjp(float4 g, float4 a, const Radii& R) {
  float4 o;
  if (KIND == K1I) {
    const float n2 = fmaf(g.x, g.x, fmaf(g.y, g.y, fmaf(g.z, g.z, g.w * g.w)));
    const float s = fminf(1.0f, rsq(n2));
    if (s < 1.0f) {
      const float d = (g.x * a.x + g.y * a.y + g.z * a.z + g.w * a.w) * (s * s);
      o = make_float4(s * (a.x - g.x * d), s * (a.y - g.y * d), s * (a.z - g.z * d), s * (a.w - g.w * d));
    } else {
      o = a;
    }
  } else if (KIND == K1A) {
    const float s1 = fminf(1.0f, rsq(fmaf(g.x, g.x, g.y * g.y)));
    const float s2 = fminf(1.0f, rsq(fmaf(g.z, g.z, g.w * g.w)));
    ball_vjp2(g.x, g.y, a.x, a.y, s1, 1.0f, o.x, o.y);
    ball_vjp2(g.z, g.w, a.z, a.w, s2, 1.0f, o.z, o.w);
  } else if (KIND == K2I) {
    const float fr = fminf(1.0f, R.ra * rsq(fmaf(g.x, g.x, g.z * g.z)));
    const float fs = fminf(1.0f, R.sa * rsq(fmaf(g.y, g.y, g.w * g.w)));
    ball_vjp2(g.x, g.z, a.x, a.z, fr, R.ra, o.x, o.z);
    ball_vjp2(g.y, g.w, a.y, a.w, fs, R.sa, o.y, o.w);
  } else {
    o.x = (R.ra > 0.0f && fabsf(g.x) <= R.ra) ? a.x : 0.0f;
    o.z = (R.ra > 0.0f && fabsf(g.z) <= R.ra) ? a.z : 0.0f;
    o.y = (R.sa > 0.0f && fabsf(g.y) <= R.sa) ? a.y : 0.0f;
    o.w = (R.sa > 0.0f && fabsf(g.w) <= R.sa) ? a.w : 0.0f;
  }
  return o;
}

struct AdjJob {
  const float2* b;
  const uint8_t* mask;
  // r_k plane of each fused step (nullptr = zero, i.e. r_1 = q_0 = 0); the
  // output step reads q_K through r[0]. The step loop is unrolled, so both
  // arrays are indexed with constants and stay in scalar registers.
  const float4* r[kMaxRev];
  const float4* adj_in;      // [2][m][n]: A then B
  float4* adj_out;           // [2][m][n] or nullptr (after the last reverse step)
  float2* gb;                // grad_b, read-modify-write
  double* lam_acc;           // per-tile accumulator slot
  int m, n, tx, ty;
  int steps;                 // reverse steps fused in this launch
  float lam, c, cc;          // lambda, 1/(8 lambda), 1/(8 lambda^2)
  float beta[kMaxRev];       // beta_{k-1} of each fused step
  Radii R;
};

__device__ __forceinline__ double block_sum_d(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// J.steps reverse steps k, k-1, ... on one tile with halo H >= steps + 1: a step
// reads (A, B) one pixel and r_k two pixels around each point it updates, so
// the valid part of the tile shrinks by one pixel per side and step. (A, B) and
// the running bbar (started from grad_b, so the sum is taken in the same order
// as one step per launch) stay in registers between steps and are stored once,
// for the tile's output pixels.
template <int KIND, int CONSTR, bool MASK, int NW, int P, bool BORDER>
__device__ __forceinline__ void adj_tile(const AdjJob& J, const int H, float2* sX1, float2* sX2, float2* sX3,
                                         float2* sX4, double* red) {
  constexpr int RH = NW * P;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c0 = J.tx * (kRW - 2 * H) - H, r0 = J.ty * (RH - 2 * H) - H;
  const int k = c0 + lane;
  const int jb = r0 + wave * P;
  const bool kin = !BORDER || (k >= 0 && k < J.n);
  const bool has_left = !BORDER || k > 0;
  const bool has_right = !BORDER || k < J.n - 1;
  const long long plane = (long long)J.m * J.n;
  const float2 z2 = make_float2(0.0f, 0.0f);
  const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);

  float4 A[P], B[P];
  float2 b[P], bacc[P];
  bool inside[P], in[P], out[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int j = jb + i;
    const int ry = wave * P + i;
    in[i] = kin && (!BORDER || (j >= 0 && j < J.m));
    out[i] = in[i] && ry >= H && ry < RH - H && lane >= H && lane < kRW - H;
    A[i] = z4;
    B[i] = z4;
    b[i] = z2;
    bacc[i] = z2;
    inside[i] = !BORDER;
    if (in[i]) {
      const long long p = (long long)j * J.n + k;
      b[i] = J.b[p];
      A[i] = J.adj_in[p];
      B[i] = J.adj_in[plane + p];
      inside[i] = MASK ? (J.mask[p] != 0) : true;
      if (out[i]) bacc[i] = J.gb[p];
    }
  }
  double lam_part = 0.0;

#pragma unroll
  for (int st = 0; st < kMaxRev; ++st) {
    if (st >= J.steps) break;
    const float4* __restrict__ rk = J.r[st];
    float4 r[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      r[i] = z4;
      if (rk && in[i]) r[i] = rk[(long long)(jb + i) * J.n + k];
    }
    // stage 1: w, y from r (up / left)
    sX1[wave * kRW + lane] = make_float2(r[P - 1].x, r[P - 1].y);
    __syncthreads();
    float2 w[P], y[P], dd[P];
    float s[P];
    {
      const float2 up_l = sX1[(wave > 0 ? wave - 1 : 0) * kRW + lane];
      const float2 up0 = (wave > 0) ? up_l : z2;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int j = jb + i;
        const float lx = from_left(r[i].z), ly = from_left(r[i].w);
        float2 up = (i > 0) ? make_float2(r[i - 1].x, r[i - 1].y) : up0;
        float2 left = make_float2(lx, ly);
        if (BORDER) {
          up = (j > 0) ? up : z2;
          left = has_left ? left : z2;
        }
        dd[i] = make_float2((r[i].x - up.x) + (r[i].z - left.x), (r[i].y - up.y) + (r[i].w - left.y));
        w[i] = dual_to_primal(b[i], r[i], up, left, J.lam);
        y[i] = proj_c_s<CONSTR>(w[i], inside[i], s[i]);
      }
    }
    // stage 2: g from y (down / right); gbar = J_PS^T A
    sX2[wave * kRW + lane] = y[0];
    __syncthreads();
    float4 gbar[P];
    {
      const float2 dn_l = sX2[(wave < NW - 1 ? wave + 1 : wave) * kRW + lane];
      const float2 down_last = (wave < NW - 1) ? dn_l : y[P - 1];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int j = jb + i;
        const bool has_down = !BORDER || j < J.m - 1;
        const float rx = from_right(y[i].x), ry = from_right(y[i].y);
        const float2 down = (i < P - 1) ? y[i + 1] : down_last;
        const float4 g = dual_step(r[i], y[i], down, make_float2(rx, ry), J.c, has_down, has_right);
        float4 gb = proj_s_vjp<KIND>(g, A[i], J.R);
        if (BORDER) {
          if (!has_down) gb.x = gb.y = 0.0f;
          if (!has_right) gb.z = gb.w = 0.0f;
        }
        gbar[i] = gb;
        if (out[i]) {
          const float l1x = has_down ? y[i].x - down.x : 0.0f, l1y = has_down ? y[i].y - down.y : 0.0f;
          const float l2x = has_right ? y[i].x - rx : 0.0f, l2y = has_right ? y[i].y - ry : 0.0f;
          lam_part += (double)(-J.cc * (gb.x * l1x + gb.y * l1y + gb.z * l2x + gb.w * l2y));
        }
      }
    }
    // stage 3: ybar = c L^T(gbar) (up / left); wbar = J_PC^T ybar
    sX3[wave * kRW + lane] = make_float2(gbar[P - 1].x, gbar[P - 1].y);
    __syncthreads();
    float2 wbar[P];
    {
      const float2 up_l = sX3[(wave > 0 ? wave - 1 : 0) * kRW + lane];
      const float2 up0 = (wave > 0) ? up_l : z2;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int j = jb + i;
        const float lx = from_left(gbar[i].z), ly = from_left(gbar[i].w);
        float2 up = (i > 0) ? make_float2(gbar[i - 1].x, gbar[i - 1].y) : up0;
        float2 left = make_float2(lx, ly);
        if (BORDER) {
          up = (j > 0) ? up : z2;
          left = has_left ? left : z2;
        }
        const float2 yb = make_float2(J.c * ((gbar[i].x - up.x) + (gbar[i].z - left.x)),
                                      J.c * ((gbar[i].y - up.y) + (gbar[i].w - left.y)));
        wbar[i] = proj_c_vjp<CONSTR>(w[i], s[i], inside[i], yb);
        bacc[i] = make_float2(bacc[i].x + wbar[i].x, bacc[i].y + wbar[i].y);
        if (out[i]) lam_part += (double)(-(wbar[i].x * dd[i].x + wbar[i].y * dd[i].y));
      }
    }
    // stage 4: rbar = gbar - lambda L(wbar) (down / right); A' = B + (1 + beta) rbar, B' = -beta rbar
    sX4[wave * kRW + lane] = wbar[0];
    __syncthreads();
    {
      const float2 dn_l = sX4[(wave < NW - 1 ? wave + 1 : wave) * kRW + lane];
      const float2 down_last = (wave < NW - 1) ? dn_l : wbar[P - 1];
      const float beta = J.beta[st];
      const float a1 = 1.0f + beta;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int j = jb + i;
        const bool has_down = !BORDER || j < J.m - 1;
        const float rx = from_right(wbar[i].x), rv = from_right(wbar[i].y);
        const float2 down = (i < P - 1) ? wbar[i + 1] : down_last;
        const float l1x = has_down ? wbar[i].x - down.x : 0.0f, l1y = has_down ? wbar[i].y - down.y : 0.0f;
        const float l2x = has_right ? wbar[i].x - rx : 0.0f, l2y = has_right ? wbar[i].y - rv : 0.0f;
        const float4 rb = make_float4(fmaf(-J.lam, l1x, gbar[i].x), fmaf(-J.lam, l1y, gbar[i].y),
                                      fmaf(-J.lam, l2x, gbar[i].z), fmaf(-J.lam, l2y, gbar[i].w));
        A[i] = make_float4(fmaf(a1, rb.x, B[i].x), fmaf(a1, rb.y, B[i].y), fmaf(a1, rb.z, B[i].z),
                           fmaf(a1, rb.w, B[i].w));
        B[i] = make_float4(-beta * rb.x, -beta * rb.y, -beta * rb.z, -beta * rb.w);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (out[i]) {
      const long long p = (long long)(jb + i) * J.n + k;
      J.gb[p] = bacc[i];
      if (J.adj_out) {
        J.adj_out[p] = A[i];
        J.adj_out[plane + p] = B[i];
      }
    }
  }
  const double tot = block_sum_d(lam_part, red);
  if (threadIdx.x == 0) *J.lam_acc += tot;
}

// Output step: w = b - lambda L^T q_K, wbar = J_PC(w)^T xbar, bbar = wbar,
// A = qbar_K = -lambda L(wbar), B = 0, lambdabar = -<wbar, L^T q_K>.
template <int CONSTR, bool MASK, int NW, int P, bool BORDER>
__device__ __forceinline__ void adj_out_tile(const AdjJob& J, const int H, const float2* __restrict__ xbar,
                                             float2* sX1, float2* sX2, double* red) {
  constexpr int RH = NW * P;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c0 = J.tx * (kRW - 2 * H) - H, r0 = J.ty * (RH - 2 * H) - H;
  const int k = c0 + lane;
  const int jb = r0 + wave * P;
  const bool kin = !BORDER || (k >= 0 && k < J.n);
  const bool has_left = !BORDER || k > 0;
  const bool has_right = !BORDER || k < J.n - 1;
  const long long plane = (long long)J.m * J.n;
  const float2 z2 = make_float2(0.0f, 0.0f);
  const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float4 q[P];
  float2 b[P], xb[P];
  bool inside[P], in[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int j = jb + i;
    in[i] = kin && (!BORDER || (j >= 0 && j < J.m));
    q[i] = z4;
    b[i] = z2;
    xb[i] = z2;
    inside[i] = !BORDER;
    if (in[i]) {
      const long long p = (long long)j * J.n + k;
      b[i] = J.b[p];
      q[i] = J.r[0][p];  // q_K plane
      xb[i] = xbar[p];
      inside[i] = MASK ? (J.mask[p] != 0) : true;
    }
  }
  sX1[wave * kRW + lane] = make_float2(q[P - 1].x, q[P - 1].y);
  __syncthreads();
  float2 wbar[P];
  double lam_part = 0.0;
  {
    const float2 up_l = sX1[(wave > 0 ? wave - 1 : 0) * kRW + lane];
    const float2 up0 = (wave > 0) ? up_l : z2;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int j = jb + i;
      const float lx = from_left(q[i].z), ly = from_left(q[i].w);
      float2 up = (i > 0) ? make_float2(q[i - 1].x, q[i - 1].y) : up0;
      float2 left = make_float2(lx, ly);
      if (BORDER) {
        up = (j > 0) ? up : z2;
        left = has_left ? left : z2;
      }
      const float2 d = make_float2((q[i].x - up.x) + (q[i].z - left.x), (q[i].y - up.y) + (q[i].w - left.y));
      const float2 w = dual_to_primal(b[i], q[i], up, left, J.lam);
      float s;
      (void)proj_c_s<CONSTR>(w, inside[i], s);
      wbar[i] = proj_c_vjp<CONSTR>(w, s, inside[i], xb[i]);
      const int ry = wave * P + i;
      if (ry >= H && ry < RH - H && lane >= H && lane < kRW - H && in[i])
        lam_part += (double)(-(wbar[i].x * d.x + wbar[i].y * d.y));
    }
  }
  sX2[wave * kRW + lane] = wbar[0];
  __syncthreads();
  {
    const float2 dn_l = sX2[(wave < NW - 1 ? wave + 1 : wave) * kRW + lane];
    const float2 down_last = (wave < NW - 1) ? dn_l : wbar[P - 1];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int j = jb + i;
      const int ry = wave * P + i;
      const bool has_down = !BORDER || j < J.m - 1;
      const float rx = from_right(wbar[i].x), rv = from_right(wbar[i].y);
      const float2 down = (i < P - 1) ? wbar[i + 1] : down_last;
      const float l1x = has_down ? wbar[i].x - down.x : 0.0f, l1y = has_down ? wbar[i].y - down.y : 0.0f;
      const float l2x = has_right ? wbar[i].x - rx : 0.0f, l2y = has_right ? wbar[i].y - rv : 0.0f;
      if (ry >= H && ry < RH - H && lane >= H && lane < kRW - H && in[i]) {
        const long long p = (long long)j * J.n + k;
        J.gb[p] = wbar[i];
        J.adj_out[p] = make_float4(-J.lam * l1x, -J.lam * l1y, -J.lam * l2x, -J.lam * l2y);
        J.adj_out[plane + p] = z4;
      }
    }
  }
  const double tot = block_sum_d(lam_part, red);
  if (threadIdx.x == 0) *J.lam_acc = tot;
}

constexpr int kNW = 8, kP = 4;

// Returns false for a workgroup with no tile (live-tile list shorter than the grid).
__device__ __forceinline__ bool adj_job_common(const AdjStepArgs& A, int& img, AdjJob& J) {
  int t;
  if (A.live) {
    // Only the live tiles, each XCD one contiguous slice of the entries (as in
    // the forward kernels); the tile keeps its own lambda-gradient slot.
    const int L = A.live[0];
    const int total = (gridDim.x / A.tiles_per_img) * L;
    constexpr int kXcd = 8;
    const int x = blockIdx.x % kXcd, i = blockIdx.x / kXcd;
    const int q = total / kXcd, rem = total % kXcd;
    if (i >= q + (x < rem ? 1 : 0)) return false;
    const int e = x * q + (x < rem ? x : rem) + i;
    img = e / L;
    t = A.live[1 + (e - img * L)];
  } else {
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    img = tile / A.tiles_per_img;
    t = tile - img * A.tiles_per_img;
  }
  const int tile = img * A.tiles_per_img + t;
  const long long px = (long long)A.m * A.n;
  J.b = reinterpret_cast<const float2*>(A.b) + img * px;
  J.mask = A.mask;
  J.adj_out = A.adj_out ? reinterpret_cast<float4*>(A.adj_out) + img * 2 * px : nullptr;
  J.gb = reinterpret_cast<float2*>(A.grad_b) + img * px;
  J.lam_acc = A.lam_acc + tile;
  J.m = A.m;
  J.n = A.n;
  J.ty = t / A.tiles_x;
  J.tx = t - J.ty * A.tiles_x;
  J.lam = A.lam[img];
  J.c = A.c[img];
  J.cc = A.cc[img];
  J.R = A.R;
  J.steps = A.steps;
  return true;
}

// Occupancy pinned at 4 waves per SIMD: left free, the type-1a and type-2i
// variants with the modulus bound take a few registers more and drop to 3.
template <int KIND, int CONSTR, bool MASK>
__global__ __launch_bounds__(kNW * 64) __attribute__((amdgpu_waves_per_eu(4))) void adj_step_kernel(AdjStepArgs A) {
  __shared__ float2 sX1[kNW * kRW], sX2[kNW * kRW], sX3[kNW * kRW], sX4[kNW * kRW];
  __shared__ double red[kNW];
  int img;
  AdjJob J;
  if (!adj_job_common(A, img, J)) return;
  const long long px = (long long)A.m * A.n;
  // plane 1 (r) of each step's state
  auto rplane = [&](const float* r) { return r ? reinterpret_cast<const float4*>(r) + img * 2 * px + px : nullptr; };
#pragma unroll
  for (int st = 0; st < kMaxRev; ++st) {
    J.r[st] = rplane(A.r[st]);
    J.beta[st] = A.beta[st];
  }
  J.adj_in = reinterpret_cast<const float4*>(A.adj_in) + img * 2 * px;
  const int H = A.halo;
  const int c0 = J.tx * (kRW - 2 * H) - H, r0 = J.ty * (kNW * kP - 2 * H) - H;
  const bool interior = c0 >= 1 && c0 + kRW <= J.n - 1 && r0 >= 1 && r0 + kNW * kP <= J.m - 1;
  if (interior)
    adj_tile<KIND, CONSTR, MASK, kNW, kP, false>(J, H, sX1, sX2, sX3, sX4, red);
  else
    adj_tile<KIND, CONSTR, MASK, kNW, kP, true>(J, H, sX1, sX2, sX3, sX4, red);
}

template <int CONSTR, bool MASK>
__global__ __launch_bounds__(kNW * 64) void adj_output_kernel(AdjStepArgs A) {
  __shared__ float2 sX1[kNW * kRW], sX2[kNW * kRW];
  __shared__ double red[kNW];
  int img;
  AdjJob J;
  if (!adj_job_common(A, img, J)) return;
  const long long px = (long long)A.m * A.n;
  J.r[0] = reinterpret_cast<const float4*>(A.r[0]) + img * 2 * px;  // plane 0 (q_K) of the final state
  J.adj_in = nullptr;
  const float2* xbar = reinterpret_cast<const float2*>(A.grad_x) + img * px;
  const int H = A.halo;
  const int c0 = J.tx * (kRW - 2 * H) - H, r0 = J.ty * (kNW * kP - 2 * H) - H;
  const bool interior = c0 >= 1 && c0 + kRW <= J.n - 1 && r0 >= 1 && r0 + kNW * kP <= J.m - 1;
  if (interior)
    adj_out_tile<CONSTR, MASK, kNW, kP, false>(J, H, xbar, sX1, sX2, red);
  else
    adj_out_tile<CONSTR, MASK, kNW, kP, true>(J, H, xbar, sX1, sX2, red);
}

// lambda = 0 or K = 0: x = P_C(b), so bbar = J_PC(b)^T xbar.
template <int CONSTR>
__global__ __launch_bounds__(256) void pc_vjp_kernel(const float2* __restrict__ b, const uint8_t* __restrict__ mask,
                                                     const float2* __restrict__ xbar, float2* __restrict__ gb,
                                                     long long px, long long total) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const bool in = mask ? (mask[i % px] != 0) : true;
  float s;
  (void)proj_c_s<CONSTR>(b[i], in, s);
  gb[i] = proj_c_vjp<CONSTR>(b[i], s, in, xbar[i]);
}

// One wave per image: lane l sums the tiles l, l + 64, ... in order, then the
// lanes are combined by a fixed butterfly, so the summation order (and the
// result) is the same on every run.
__global__ __launch_bounds__(64) void lam_final_kernel(const double* __restrict__ acc, int tiles_per_img,
                                                       int batch, float* __restrict__ out) {
  const int img = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int t = lane; t < tiles_per_img; t += 64) s += acc[(long long)img * tiles_per_img + t];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0 && img < batch) out[img] = (float)s;
}

}  // namespace

int adj_tile_rows() { return kNW * kP; }

hipError_t launch_adj_step(const AdjStepArgs& a, int kind, int constr, int batch, hipStream_t s) {
  const int nb = a.tiles_per_img * batch;
  const bool mask = a.mask != nullptr;
#define CTV_ADJ(KI)                                                                                     \
  if (constr == C_MOD) {                                                                                \
    if (mask) hipLaunchKernelGGL((adj_step_kernel<KI, C_MOD, true>), dim3(nb), dim3(kNW * 64), 0, s, a);  \
    else hipLaunchKernelGGL((adj_step_kernel<KI, C_MOD, false>), dim3(nb), dim3(kNW * 64), 0, s, a);      \
  } else {                                                                                              \
    if (mask) hipLaunchKernelGGL((adj_step_kernel<KI, C_NONE, true>), dim3(nb), dim3(kNW * 64), 0, s, a); \
    else hipLaunchKernelGGL((adj_step_kernel<KI, C_NONE, false>), dim3(nb), dim3(kNW * 64), 0, s, a);     \
  }
  switch (kind) {
    case K1I: CTV_ADJ(K1I) break;
    case K1A: CTV_ADJ(K1A) break;
    case K2I: CTV_ADJ(K2I) break;
    default: CTV_ADJ(K2A) break;
  }
#undef CTV_ADJ
  return hipGetLastError();
}

hipError_t launch_adj_output(const AdjStepArgs& a, int constr, int batch, hipStream_t s) {
  const int nb = a.tiles_per_img * batch;
  const bool mask = a.mask != nullptr;
  if (constr == C_MOD) {
    if (mask) hipLaunchKernelGGL((adj_output_kernel<C_MOD, true>), dim3(nb), dim3(kNW * 64), 0, s, a);
    else hipLaunchKernelGGL((adj_output_kernel<C_MOD, false>), dim3(nb), dim3(kNW * 64), 0, s, a);
  } else {
    if (mask) hipLaunchKernelGGL((adj_output_kernel<C_NONE, true>), dim3(nb), dim3(kNW * 64), 0, s, a);
    else hipLaunchKernelGGL((adj_output_kernel<C_NONE, false>), dim3(nb), dim3(kNW * 64), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_pc_vjp(const float* b, const uint8_t* mask, const float* xbar, float* gb, long long px, int batch,
                         int constr, hipStream_t s) {
  const long long total = px * batch;
  const int nb = (int)((total + 255) / 256);
  const float2* b2 = reinterpret_cast<const float2*>(b);
  const float2* x2 = reinterpret_cast<const float2*>(xbar);
  float2* g2 = reinterpret_cast<float2*>(gb);
  if (constr == C_MOD)
    hipLaunchKernelGGL(pc_vjp_kernel<C_MOD>, dim3(nb), dim3(256), 0, s, b2, mask, x2, g2, px, total);
  else
    hipLaunchKernelGGL(pc_vjp_kernel<C_NONE>, dim3(nb), dim3(256), 0, s, b2, mask, x2, g2, px, total);
  return hipGetLastError();
}

hipError_t launch_lam_final(const double* acc, int tiles_per_img, int batch, float* out, hipStream_t s) {
  hipLaunchKernelGGL(lam_final_kernel, dim3((unsigned)batch), dim3(64), 0, s, acc, tiles_per_img, batch, out);
  return hipGetLastError();
}

}  // namespace ctv

namespace ctv {
namespace {
__global__ __launch_bounds__(256) void zero_f32_kernel(float* __restrict__ p, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0f;
}
}  // namespace

hipError_t launch_zero_f32(float* p, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}
}  // namespace ctv
