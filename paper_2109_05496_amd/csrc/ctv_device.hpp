// Per-pixel operators of the complex constrained TV solver, shared by every
// kernel of the HIP path (plain, batched, adjoint) so that they all perform the
// same float32 operations in the same order and agree bit for bit.
//
// Data layout (padded): the dual variable of a pixel is one float4
// (r1, s1, r2, s2): the vertical difference pair Q1 = r1 + i s1 and the
// horizontal pair Q2 = r2 + i s2 (Proposition 1's q = (r1, r2, s1, s2)).
// Q1 on the last row and Q2 on the last column do not exist in the paper; they
// are held at exactly 0, which makes the paper's separate boundary formulas
// (Eqs. 17, 20, 34, 35) coincide with the interior ones.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctv_types.hpp"

namespace ctv {

// Hardware reciprocal square root (v_rsq_f32, ~1 ulp). Its arguments here are
// sums of squares: a denormal argument is read as 0 and gives +inf, which the
// callers' min(1, .) maps to a unit scale - the right answer for a vector that
// small.
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// P_C of one pixel: x / max{1, |x|} (Eq. 26) when the modulus constraint is
// on, then forced to 0 outside the support (a zero scale; adding +0 to the
// product turns -0 into +0, so masked pixels hold exactly +0 whatever the sign
// of w, and a tile that is never computed matches one that is).
template <int CONSTR>
__device__ __forceinline__ float2 proj_c(float2 w, bool inside) {
  float2 y = w;
  if (CONSTR == C_MOD) {
    const float n2 = fmaf(w.x, w.x, w.y * w.y);
    float s = fminf(1.0f, rsq(n2));  // 1/max{1,|w|}; rsqrt(0) = inf gives 1
    s = inside ? s : 0.0f;
    y.x = fmaf(w.x, s, 0.0f);  // the product, with +0 in place of -0
    y.y = fmaf(w.y, s, 0.0f);
  } else {
    y.x = inside ? w.x : 0.0f;
    y.y = inside ? w.y : 0.0f;
  }
  return y;
}

// P_S of one pixel's dual group(s), as the scale applied to each entry of g:
//   1i: the 4-vector onto the unit ball (Eq. 20)
//   1a: each complex direction pair onto the unit disc (Eq. 33)
//   2i: (r1, r2) onto the alpha-disc, (s1, s2) onto the (1-alpha)-disc (Eq. 35)
// Each scale is min(1, radius / norm), i.e. the paper's radius / max{radius, norm}.
// Type 2a (Eq. 37) clips each real entry to [-alpha, alpha] or
// [-(1-alpha), 1-alpha] instead and has no scale form.
template <int KIND>
__device__ __forceinline__ float4 ps_scale(float4 g, const Radii& R) {
  if (KIND == K1I) {
    const float n2 = fmaf(g.x, g.x, fmaf(g.y, g.y, fmaf(g.z, g.z, g.w * g.w)));
    const float s = fminf(1.0f, rsq(n2));
    return make_float4(s, s, s, s);
  } else if (KIND == K1A) {
    const float n1 = fmaf(g.x, g.x, g.y * g.y);
    const float n2 = fmaf(g.z, g.z, g.w * g.w);
    const float s1 = fminf(1.0f, rsq(n1));
    const float s2 = fminf(1.0f, rsq(n2));
    return make_float4(s1, s1, s2, s2);
  } else {
    // rho / max{rho, ||v||} = min(1, rho / ||v||); a zero radius gives 0 * inf = NaN
    // at v = 0, which fminf turns into 1, and 0 * v = 0 either way.
    const float nr = fmaf(g.x, g.x, g.z * g.z);
    const float ns = fmaf(g.y, g.y, g.w * g.w);
    const float fr = fminf(1.0f, R.ra * rsq(nr));
    const float fs = fminf(1.0f, R.sa * rsq(ns));
    return make_float4(fr, fs, fr, fs);
  }
}

// One dual update in place: q <- P_S(g) (q_k of Algorithm 2, line 4) and
// r <- q_k + beta_k (q_k - q_{k-1}) (line 5), with q holding q_{k-1} on entry.
// The difference d = P_S(g) - q_{k-1} is formed first (one fused multiply-add
// per entry for the scaled kinds) and q_k = q_{k-1} + d, so the update writes
// q's registers in place: three operations per entry, and q_k within a
// rounding of P_S(g).
template <int KIND>
__device__ __forceinline__ void dual_update(float4 g, const Radii& R, float beta, float4& q, float4& r) {
  float dx, dy, dz, dw;
  if (KIND == K2A) {
    dx = fminf(fmaxf(g.x, -R.ra), R.ra) - q.x;
    dy = fminf(fmaxf(g.y, -R.sa), R.sa) - q.y;
    dz = fminf(fmaxf(g.z, -R.ra), R.ra) - q.z;
    dw = fminf(fmaxf(g.w, -R.sa), R.sa) - q.w;
  } else {
    const float4 s = ps_scale<KIND>(g, R);
    dx = fmaf(g.x, s.x, -q.x);
    dy = fmaf(g.y, s.y, -q.y);
    dz = fmaf(g.z, s.z, -q.z);
    dw = fmaf(g.w, s.w, -q.w);
  }
  q = make_float4(q.x + dx, q.y + dy, q.z + dz, q.w + dw);
  r = make_float4(fmaf(beta, dx, q.x), fmaf(beta, dy, q.y), fmaf(beta, dz, q.z), fmaf(beta, dw, q.w));
}

// w = b - lambda * L^T(r) at one pixel, per channel
//   (L^T a)_{j,k} = a1_{j,k} - a1_{j-1,k} + a2_{j,k} - a2_{j,k-1},
// the adjoint of the forward differences of Eqs. (5)-(6); `up` is the (r1, s1)
// pair of pixel (j-1, k) and `left` the (r2, s2) pair of (j, k-1), both zero
// outside the image.
__device__ __forceinline__ float2 dual_to_primal(float2 b, float4 r, float2 up, float2 left,
                                                 float lam) {
  const float du = (r.x - up.x) + (r.z - left.x);
  const float dv = (r.y - up.y) + (r.w - left.y);
  return make_float2(fmaf(-lam, du, b.x), fmaf(-lam, dv, b.y));
}

// g = r + L(y) / (8 lambda): the dual gradient step of Algorithm 2, line 3,
// with grad h from Eq. (19) and step 1/(16 lambda^2). `down` is y at (j+1, k),
// `right` y at (j, k+1); the differences that do not exist (last row /
// last column) are kept at zero.
__device__ __forceinline__ float4 dual_step(float4 r, float2 y, float2 down, float2 right,
                                            float c, bool has_down, bool has_right) {
  float4 g;
  g.x = has_down ? fmaf(c, y.x - down.x, r.x) : 0.0f;
  g.y = has_down ? fmaf(c, y.y - down.y, r.y) : 0.0f;
  g.z = has_right ? fmaf(c, y.x - right.x, r.z) : 0.0f;
  g.w = has_right ? fmaf(c, y.y - right.y, r.w) : 0.0f;
  return g;
}

// Streaming (non-temporal) stores, used for the forward tile's dual state and
// x: they leave less dirty data in the L2 caches to be written back at the
// kernel boundary (measured: +2 % at 2048^2). Loads keep the default policy,
// since a tile's halo is re-read by its neighbours through L2; the r history
// and the adjoint state, re-read soon by the same XCD, measured slower when
// streamed and keep plain stores.
__device__ __forceinline__ void store_nt(float4* p, float4 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
  __builtin_nontemporal_store(v.z, &p->z);
  __builtin_nontemporal_store(v.w, &p->w);
}
__device__ __forceinline__ void store_nt(float2* p, float2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

// Consecutive workgroup ids are spread round-robin over the 8 XCDs of an
// MI355X; give each XCD one contiguous range of tiles so neighbouring tiles
// (which re-read each other's halos) share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int q = nblocks / kXcd, rem = nblocks % kXcd;
  const int x = bid % kXcd, i = bid / kXcd;
  return x * q + (x < rem ? x : rem) + i;
}

}  // namespace ctv
