// Forward FGP kernels for gfx950: several iterations of Algorithm 2 fused per
// launch on LDS-staged tiles with a halo, the output step of Eq. (18), the
// projection-only path, and the duality-gap reduction.
//
// Tile scheme: a workgroup of 256 threads (4 wave64s) owns a region of 64
// columns x RH rows. Lane l holds column l; wave w holds rows w, w+4, w+8, ...
// Each thread keeps its pixels' b, q_k and r_{k+1} in registers. One iteration:
//   1. publish r (as the (r1,s1) and (r2,s2) pairs) to LDS;           barrier
//   2. y = P_C(b - lambda L^T r) using the up / left neighbours; y -> LDS; barrier
//   3. g = r + L(y)/(8 lambda) using the down / right neighbours,
//      q' = P_S(g), r' = q' + beta (q' - q).
// Values near the region edge go stale by one pixel per iteration, so after T
// fused iterations the central (64 - 2H) x (RH - 2H) pixels are exact when the
// halo H >= T (H >= T + 1 when the Eq. (18) epilogue runs in the same launch,
// since x reads q one pixel up and left). Image borders are exact at any
// distance: the differences that leave the image are zero by construction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ctv_device.hpp"
#include "ctv_kernels.hpp"
#include "ctv_tile.hpp"

namespace ctv {


constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;


template <int KIND, int CONSTR, bool MASK, int RH>
__device__ __forceinline__ void fgp_tile(const TileJob& J, const int H, const float* sBeta,
                                         float2* __restrict__ sA1, float2* __restrict__ sA2,
                                         float2* __restrict__ sY) {
  constexpr int PPT = RH / kWaves;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int OW = kRW - 2 * H, OH = RH - 2 * H;
  const int c0 = J.tx * OW - H, r0 = J.ty * OH - H;
  const int k = c0 + lane;
  const bool kin = (k >= 0) && (k < J.n);
  const bool has_left = k > 0;
  const bool has_right = k < J.n - 1;
  const long long plane = (long long)J.m * J.n;
  const float2 zero2 = make_float2(0.0f, 0.0f);

  float4 q[PPT], r[PPT];
  float2 b[PPT];
  bool inside[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int j = r0 + wave + kWaves * i;
    const bool in = kin && j >= 0 && j < J.m;
    q[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    r[i] = q[i];
    b[i] = zero2;
    inside[i] = false;
    if (in) {
      const long long p = (long long)j * J.n + k;
      b[i] = J.b[p];
      if (J.st_in) {
        q[i] = J.st_in[p];
        r[i] = J.st_in[plane + p];
      }
      inside[i] = MASK ? (J.mask[p] != 0) : true;
    }
  }

  for (int it = 0; it < J.T; ++it) {
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int ry = wave + kWaves * i;
      sA1[ry * kRW + lane] = make_float2(r[i].x, r[i].y);
      sA2[ry * kRW + lane] = make_float2(r[i].z, r[i].w);
    }
    __syncthreads();
    float2 y[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int ry = wave + kWaves * i;
      const int j = r0 + ry;
      const float2 up = (j > 0) ? sA1[(ry > 0 ? ry - 1 : 0) * kRW + lane] : zero2;
      const float2 left = has_left ? sA2[ry * kRW + (lane > 0 ? lane - 1 : 0)] : zero2;
      y[i] = proj_c<CONSTR>(dual_to_primal(b[i], r[i], up, left, J.lam), inside[i]);
      sY[ry * kRW + lane] = y[i];
    }
    __syncthreads();
    const float beta = sBeta[it];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int ry = wave + kWaves * i;
      const int j = r0 + ry;
      const float2 down = sY[(ry < RH - 1 ? ry + 1 : RH - 1) * kRW + lane];
      const float2 right = sY[ry * kRW + (lane < kRW - 1 ? lane + 1 : kRW - 1)];
      const float4 g = dual_step(r[i], y[i], down, right, J.c, j < J.m - 1, has_right);
      dual_update<KIND>(g, J.R, beta, q[i], r[i]);
    }
  }

  const bool col_out = lane >= H && lane < kRW - H && kin;
  if (J.x) {
    // Eq. (18): x = P_C(b - lambda L^T q_K). The LDS pairs were last read in
    // step 2 of the final iteration, which a barrier has already closed.
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int ry = wave + kWaves * i;
      sA1[ry * kRW + lane] = make_float2(q[i].x, q[i].y);
      sA2[ry * kRW + lane] = make_float2(q[i].z, q[i].w);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int ry = wave + kWaves * i;
      const int j = r0 + ry;
      if (col_out && ry >= H && ry < RH - H && j < J.m) {
        const float2 up = (j > 0) ? sA1[(ry - 1) * kRW + lane] : zero2;
        const float2 left = has_left ? sA2[ry * kRW + lane - 1] : zero2;
        J.x[(long long)j * J.n + k] =
            proj_c<CONSTR>(dual_to_primal(b[i], q[i], up, left, J.lam), inside[i]);
      }
    }
  }
  if (J.st_out) {
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int ry = wave + kWaves * i;
      const int j = r0 + ry;
      if (col_out && ry >= H && ry < RH - H && j < J.m) {
        const long long p = (long long)j * J.n + k;
        J.st_out[p] = q[i];
        J.st_out[plane + p] = r[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column-register tile. A workgroup of NW wave64s owns 64 columns x NW*P rows;
// lane l holds column l and wave w the P consecutive rows [w*P, (w+1)*P).
// Vertical neighbours are in the thread's own registers; horizontal ones come
// from the adjacent lane through DPP whole-wave shifts; only the rows at the
// boundary between two waves go through LDS (one row of (r1,s1) down, one row
// of y up per iteration). Same arithmetic, same halo rule as above.
// ---------------------------------------------------------------------------

// Dual-state element access. COH = true (the dataflow kernel) uses 64-bit
// agent-scope atomic accesses, which are coherent across the XCDs' separate
// L2 caches without any cache-wide write-back or invalidate.
template <bool COH>
__device__ __forceinline__ float4 ld_state(const float4* p) {
  if (!COH) return *p;
  unsigned long long* u = reinterpret_cast<unsigned long long*>(const_cast<float4*>(p));
  const unsigned long long a = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(u + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_float4(__uint_as_float((unsigned)a), __uint_as_float((unsigned)(a >> 32)),
                     __uint_as_float((unsigned)b), __uint_as_float((unsigned)(b >> 32)));
}
template <bool COH>
__device__ __forceinline__ void st_state(float4* p, float4 v) {
  if (!COH) {
    store_nt(p, v);
    return;
  }
  unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
  const unsigned long long a = (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
  const unsigned long long b = (unsigned long long)__float_as_uint(v.z) | ((unsigned long long)__float_as_uint(v.w) << 32);
  __hip_atomic_store(u, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(u + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// BORDER = false is the fast path for tiles whose region lies at least one
// pixel inside the image on every side: no neighbour there leaves the image, so
// the boundary selects disappear. Rows are skipped once they fall outside the
// part of the region that can still reach the output (the shrinking trapezoid
// of the fused iterations); one row more than the q rows needs y.
template <int KIND, int CONSTR, bool MASK, int NW, int P, bool BORDER, bool HIST = false, bool COH = false>
__device__ __forceinline__ void fgp_tile_col(const TileJob& J, const int H, const float* sBeta,
                                             float2* __restrict__ sBot, float2* __restrict__ sTop) {
  constexpr int RH = NW * P;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int OW = kRW - 2 * H, OH = RH - 2 * H;
  const int c0 = J.tx * OW - H, r0 = J.ty * OH - H;
  const int k = c0 + lane;
  const int jb = r0 + wave * P;
  const bool kin = !BORDER || ((k >= 0) && (k < J.n));
  const bool has_left = !BORDER || k > 0;
  const bool has_right = !BORDER || k < J.n - 1;
  const long long plane = (long long)J.m * J.n;
  const float2 zero2 = make_float2(0.0f, 0.0f);

  // Offset of the region's row i at column c0: the same for every lane of the
  // wave, so each access below is a scalar row base plus the lane's offset
  // (no per-lane 64-bit address arithmetic).
  auto row_off = [&](int i) { return (long long)(jb + i) * J.n + c0; };
  float4 q[P], r[P];
  float2 b[P];
  bool inside[P];
  if (!BORDER) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const long long o = row_off(i);
      b[i] = (J.b + o)[lane];
      inside[i] = MASK ? ((J.mask + o)[lane] != 0) : true;
    }
    if (J.st_in) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const long long o = row_off(i);
        q[i] = ld_state<COH>(J.st_in + o + lane);
        r[i] = ld_state<COH>(J.st_in + plane + o + lane);
      }
    } else {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        q[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        r[i] = q[i];
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int j = jb + i;
      const bool in = kin && j >= 0 && j < J.m;
      q[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      r[i] = q[i];
      b[i] = zero2;
      inside[i] = false;
      if (in) {
        const long long o = row_off(i);
        b[i] = (J.b + o)[lane];
        if (J.st_in) {
          q[i] = ld_state<COH>(J.st_in + o + lane);
          r[i] = ld_state<COH>(J.st_in + plane + o + lane);
        }
        inside[i] = MASK ? ((J.mask + o)[lane] != 0) : true;
      }
    }
  }

  const bool col_out = lane >= H && lane < kRW - H && kin;

  // Rows whose q can still reach the output: after the last iteration the
  // stored state needs rows [H, RH-H) and Eq. (18) additionally reads q one row
  // up, so at iteration t the needed rows are [t + eu, RH - t - ed).
  const int ed = H - J.T;
  const int eu = ed - (J.x ? 1 : 0);
  float2 y[P];
#pragma unroll
  for (int i = 0; i < P; ++i) y[i] = zero2;
  for (int it = 0; it < J.T; ++it) {
    // Live rows of this wave as bit masks (uniform): y on [lo, hi], q on [lo, hi).
    const int lo = it + 1 + eu - wave * P, hi = RH - (it + 1) - ed - wave * P;
    const unsigned ym = row_bits(lo, hi + 1, P), qm = row_bits(lo, hi, P);
    sBot[wave * kRW + lane] = make_float2(r[P - 1].x, r[P - 1].y);
    __syncthreads();
    const float2 up_lds = sBot[(wave > 0 ? wave - 1 : 0) * kRW + lane];
    const float2 up0 = (wave > 0) ? up_lds : zero2;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      if (ym & (1u << i)) {
        const int j = jb + i;
        const float lx = lane_from_left(r[i].z), ly = lane_from_left(r[i].w);
        float2 up = (i > 0) ? make_float2(r[i - 1].x, r[i - 1].y) : up0;
        float2 left = make_float2(lx, ly);
        if (BORDER) {
          up = (j > 0) ? up : zero2;
          left = has_left ? left : zero2;
        }
        y[i] = proj_c<CONSTR>(dual_to_primal(b[i], r[i], up, left, J.lam), inside[i]);
      }
    }
    sTop[wave * kRW + lane] = y[0];
    __syncthreads();
    const float2 down_lds = sTop[(wave < NW - 1 ? wave + 1 : wave) * kRW + lane];
    const float2 down_last = (wave < NW - 1) ? down_lds : y[P - 1];
    const float beta = sBeta[it];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      if (qm & (1u << i)) {
        const int j = jb + i;
        const float rx = lane_from_right(y[i].x), rv = lane_from_right(y[i].y);
        const float2 down = (i < P - 1) ? y[i + 1] : down_last;
        const float4 g = dual_step(r[i], y[i], down, make_float2(rx, rv), J.c,
                                   !BORDER || j < J.m - 1, has_right);
        dual_update<KIND>(g, J.R, beta, q[i], r[i]);
      }
    }
    if (HIST) {
      // r_{k+1} of this iteration for the output part of the tile (the reverse pass reads it)
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int j = jb + i;
        const int ry = wave * P + i;
        if (col_out && ry >= H && ry < RH - H && (!BORDER || j < J.m))
          (J.r_hist + (it * J.hist_stride + row_off(i)))[lane] = r[i];
      }
    }
  }

  if (J.x) {
    sBot[wave * kRW + lane] = make_float2(q[P - 1].x, q[P - 1].y);
    __syncthreads();
    const float2 up_lds = sBot[(wave > 0 ? wave - 1 : 0) * kRW + lane];
    const float2 up0 = (wave > 0) ? up_lds : zero2;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int j = jb + i;
      const int ry = wave * P + i;
      if (ry >= H && ry < RH - H) {
        const float lx = lane_from_left(q[i].z), ly = lane_from_left(q[i].w);
        float2 up = (i > 0) ? make_float2(q[i - 1].x, q[i - 1].y) : up0;
        float2 left = make_float2(lx, ly);
        if (BORDER) {
          up = (j > 0) ? up : zero2;
          left = has_left ? left : zero2;
        }
        const float2 xv = proj_c<CONSTR>(dual_to_primal(b[i], q[i], up, left, J.lam), inside[i]);
        if (col_out && (!BORDER || j < J.m)) store_nt(J.x + row_off(i) + lane, xv);
      }
    }
  }
  if (J.st_out) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int j = jb + i;
      const int ry = wave * P + i;
      if (col_out && ry >= H && ry < RH - H && (!BORDER || j < J.m)) {
        const long long o = row_off(i);
        st_state<COH>(J.st_out + o + lane, q[i]);
        st_state<COH>(J.st_out + plane + o + lane, r[i]);
      }
    }
  }
}

// HIST: also store r after every fused iteration (the adjoint's recomputation).
template <int KIND, int CONSTR, bool MASK, int NW, int P, bool HIST = false>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void fgp_col_kernel(FgpPlainArgs P_) {
  __shared__ float2 sBot[NW * kRW];
  __shared__ float2 sTop[NW * kRW];
  __shared__ float sBeta[kMaxFuse];
  if (threadIdx.x < kMaxFuse) sBeta[threadIdx.x] = P_.beta[threadIdx.x];
  __syncthreads();
  const int per_img = P_.tiles_x * P_.tiles_y;
  int img, t;
  if (P_.live) {
    // Only the live tiles: entry e of the chunk's images x live tiles is tile
    // live[1 + e % L] of image e / L, and each XCD takes one contiguous slice of
    // the entries (equal counts, neighbouring tiles in one L2). Workgroups past
    // their XCD's slice have nothing to do.
    const int L = P_.live[0];
    const int total = (gridDim.x / per_img) * L;
    constexpr int kXcd = 8;
    const int x = blockIdx.x % kXcd, i = blockIdx.x / kXcd;
    const int q = total / kXcd, rem = total % kXcd;
    if (i >= q + (x < rem ? 1 : 0)) return;
    const int e = x * q + (x < rem ? x : rem) + i;
    img = e / L;
    t = P_.live[1 + (e - img * L)];
  } else {
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    img = tile / per_img;
    t = tile - img * per_img;
  }
  const long long px = (long long)P_.m * P_.n;
  TileJob J;
  J.b = reinterpret_cast<const float2*>(P_.b) + img * px;
  J.mask = P_.mask;
  J.st_in = P_.st_in ? reinterpret_cast<const float4*>(P_.st_in) + img * 2 * px : nullptr;
  J.st_out = P_.st_out ? reinterpret_cast<float4*>(P_.st_out) + img * 2 * px : nullptr;
  J.x = P_.x ? reinterpret_cast<float2*>(P_.x) + img * px : nullptr;
  J.m = P_.m;
  J.n = P_.n;
  J.ty = t / P_.tiles_x;
  J.tx = t - J.ty * P_.tiles_x;
  J.lam = P_.lam[img];
  J.c = P_.c[img];
  J.R = P_.R;
  J.T = P_.T;
  J.r_hist = HIST ? reinterpret_cast<float4*>(P_.r_hist) + img * 2 * px + px : nullptr;
  J.hist_stride = P_.r_hist_stride / 4;
  const int H = P_.halo;
  const int c0 = J.tx * (kRW - 2 * H) - H, r0 = J.ty * (NW * P - 2 * H) - H;
  const bool interior = c0 >= 1 && c0 + kRW <= J.n - 1 && r0 >= 1 && r0 + NW * P <= J.m - 1;
  if (interior)
    fgp_tile_col<KIND, CONSTR, MASK, NW, P, false, HIST>(J, H, sBeta, sBot, sTop);
  else
    fgp_tile_col<KIND, CONSTR, MASK, NW, P, true, HIST>(J, H, sBeta, sBot, sTop);
}

// ---------------------------------------------------------------------------
// Persistent dataflow kernel (see FgpFlowArgs). Memory ordering: the dual
// state, the only data that passes between tasks, is read and written with
// agent-scope (device-coherent) atomic accesses, which the 8 XCDs' separate L2
// caches keep coherent. A task waits for all of its own memory operations to
// complete (every wave) and crosses a workgroup barrier before raising its
// done flag; a waiting task polls its neighbours' flags with agent-scope atomic
// loads and crosses a barrier before loading. Every wait is bounded: after kFlowSpin
// polls (about a second) it records the failure in *err and proceeds, and
// every other wait then stops at its next check, so the grid always drains.
// A task that proceeds without its inputs may compute wrong values, and so may
// every task that depends on it; all of them come after the failure was
// recorded, so an epilogue task that finds *err set writes NaN into its output
// pixels of x and of the returned state instead of Eq. (18). Results are
// therefore either exact or NaN, never silently wrong.
constexpr int kFlowSpin = 1 << 20;

// NaN into the output pixels of one tile of one image (x and, if given, both
// planes of the returned state): the dataflow schedule's failure report.
__device__ void flow_fail_tile(float2* x, float4* st, int m, int n, int tx, int ty, int OW, int OH) {
  const float nan = __builtin_nanf("");
  const int k = tx * OW + (int)(threadIdx.x & 63);
  if ((int)(threadIdx.x & 63) >= OW || k >= n) return;
  const long long plane = (long long)m * n;
  for (int j = ty * OH + (int)(threadIdx.x >> 6); j < min(m, (ty + 1) * OH); j += (int)(blockDim.x >> 6)) {
    const long long p = (long long)j * n + k;
    if (x) x[p] = make_float2(nan, nan);
    if (st) {
      st[p] = make_float4(nan, nan, nan, nan);
      st[plane + p] = make_float4(nan, nan, nan, nan);
    }
  }
}

template <int KIND, int CONSTR, bool MASK>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void fgp_flow_kernel(FgpFlowArgs A) {
  constexpr int NW = 8, P = 8;
  __shared__ float2 sBot[NW * kRW];
  __shared__ float2 sTop[NW * kRW];
  __shared__ float sBeta[kMaxFuse];
  __shared__ int sTicket;
  __shared__ int sErr;
  const int per_img = A.tiles_x * A.tiles_y;
  const int per_step = per_img * A.batch;
  const int total = per_step * (A.steps + 1);
  const long long px = (long long)A.m * A.n;
  const int H = A.halo;
  if (A.preset_err && threadIdx.x == 0) __hip_atomic_store(A.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    __syncthreads();  // the previous task is done with LDS
    if (threadIdx.x == 0) sTicket = atomicAdd(A.counter, 1);
    __syncthreads();
    const int ticket = sTicket;
    if (ticket >= total) break;
    const int st = ticket / per_step;
    const int rem = ticket - st * per_step;
    const int img = rem / per_img;
    const int t = rem - img * per_img;
    const int ty = t / A.tiles_x;
    const int tx = t - ty * A.tiles_x;
    int* done_img = A.done + (long long)img * per_img;
    if (st > 0) {
      if (threadIdx.x < 9) {
        const int ny = ty + (int)threadIdx.x / 3 - 1, nx = tx + (int)threadIdx.x % 3 - 1;
        if (ny >= 0 && ny < A.tiles_y && nx >= 0 && nx < A.tiles_x) {
          const int* flag = done_img + ny * A.tiles_x + nx;
          int spins = 0;
          while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < st) {
            if (++spins > kFlowSpin) {
              __hip_atomic_store(A.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            // once any wait has given up, stop waiting everywhere so the grid drains at once
            if ((spins & 63) == 0 && __hip_atomic_load(A.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            __builtin_amdgcn_s_sleep(2);
          }
        }
      }
      __syncthreads();
    }
    const bool epi = (st == A.steps);
    const int T = epi ? 0 : (st == A.steps - 1 ? A.T_last : A.T);
    if (threadIdx.x < kMaxFuse) sBeta[threadIdx.x] = ((int)threadIdx.x < T) ? A.beta[st * A.T + threadIdx.x] : 0.0f;
    if (threadIdx.x == 0) sErr = epi ? __hip_atomic_load(A.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    __syncthreads();
    float* in_buf = (st % 2 == 0) ? A.buf0 : A.buf1;
    if (sErr) {
      // A wait gave up somewhere and this tile's output may depend on it. The
      // last chunk of a call reports it in x and the returned state; an
      // earlier chunk (no x) in the state the next chunk starts from, where
      // the NaN spreads to x.
      float4* fst = A.x ? reinterpret_cast<float4*>(A.st_out) : reinterpret_cast<float4*>(in_buf);
      flow_fail_tile(A.x ? reinterpret_cast<float2*>(A.x) + img * px : nullptr, fst ? fst + img * 2 * px : nullptr,
                     A.m, A.n, tx, ty, kRW - 2 * H, NW * P - 2 * H);
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_store(done_img + t, st + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    float* out_buf = (st % 2 == 0) ? A.buf1 : A.buf0;
    const float* src = (st == 0) ? A.st_in : in_buf;
    float* dst = epi ? A.st_out : out_buf;
    TileJob J;
    J.b = reinterpret_cast<const float2*>(A.b) + img * px;
    J.mask = A.mask;
    J.st_in = src ? reinterpret_cast<const float4*>(src) + img * 2 * px : nullptr;
    J.st_out = dst ? reinterpret_cast<float4*>(dst) + img * 2 * px : nullptr;
    J.x = (epi && A.x) ? reinterpret_cast<float2*>(A.x) + img * px : nullptr;  // no x before the last chunk
    J.m = A.m;
    J.n = A.n;
    J.ty = ty;
    J.tx = tx;
    J.lam = A.lam[img];
    J.c = A.c[img];
    J.R = A.R;
    J.T = T;
    J.r_hist = nullptr;
    J.hist_stride = 0;
    const int c0 = tx * (kRW - 2 * H) - H, r0 = ty * (NW * P - 2 * H) - H;
    const bool interior = c0 >= 1 && c0 + kRW <= J.n - 1 && r0 >= 1 && r0 + NW * P <= J.m - 1;
    if (interior)
      fgp_tile_col<KIND, CONSTR, MASK, NW, P, false, false, true>(J, H, sBeta, sBot, sTop);
    else
      fgp_tile_col<KIND, CONSTR, MASK, NW, P, true, false, true>(J, H, sBeta, sBot, sTop);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's state stores are complete (device-coherent)
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(done_img + t, st + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Whole image in one tile (see FgpSingleArgs): halo 0, every row always live.
// 16 waves x 4 rows: the same 64 x 64 region as the 8 x 8 tile with half the
// rows per wave, i.e. shorter dependent chains for this latency-bound case.
constexpr int kSingleNW = 16, kSingleP = 4;

template <int KIND, int CONSTR, bool MASK>
__global__ __launch_bounds__(kSingleNW * 64) void fgp_single_kernel(FgpSingleArgs A) {
  __shared__ float2 sBot[kSingleNW * kRW];
  __shared__ float2 sTop[kSingleNW * kRW];
  __shared__ float sBeta[kFlowMaxIters];
  for (int i = threadIdx.x; i < A.T; i += blockDim.x) sBeta[i] = A.beta[i];
  __syncthreads();
  const int img = blockIdx.x;
  const long long px = (long long)A.m * A.n;
  TileJob J;
  J.b = reinterpret_cast<const float2*>(A.b) + img * px;
  J.mask = A.mask;
  J.st_in = A.st_in ? reinterpret_cast<const float4*>(A.st_in) + img * 2 * px : nullptr;
  J.st_out = A.st_out ? reinterpret_cast<float4*>(A.st_out) + img * 2 * px : nullptr;
  J.x = A.x ? reinterpret_cast<float2*>(A.x) + img * px : nullptr;
  J.m = A.m;
  J.n = A.n;
  J.tx = 0;
  J.ty = 0;
  J.lam = A.lam[img];
  J.c = A.c[img];
  J.R = A.R;
  J.T = A.T;
  J.r_hist = nullptr;
  J.hist_stride = 0;
  fgp_tile_col<KIND, CONSTR, MASK, kSingleNW, kSingleP, true>(J, 0, sBeta, sBot, sTop);
}

// ---------------------------------------------------------------------------
// Plain kernel: `batch` images of one shape, one parameter set.
// ---------------------------------------------------------------------------
template <int KIND, int CONSTR, bool MASK, int RH>
__global__ __launch_bounds__(kThreads) void fgp_plain_kernel(FgpPlainArgs P) {
  __shared__ float2 sA1[RH * kRW];
  __shared__ float2 sA2[RH * kRW];
  __shared__ float2 sY[RH * kRW];
  __shared__ float sBeta[kMaxFuse];
  if (threadIdx.x < kMaxFuse) sBeta[threadIdx.x] = P.beta[threadIdx.x];
  __syncthreads();
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int per_img = P.tiles_x * P.tiles_y;
  const int img = tile / per_img;
  const int t = tile - img * per_img;
  const long long px = (long long)P.m * P.n;
  TileJob J;
  J.b = reinterpret_cast<const float2*>(P.b) + img * px;
  J.mask = P.mask;
  J.st_in = P.st_in ? reinterpret_cast<const float4*>(P.st_in) + img * 2 * px : nullptr;
  J.st_out = P.st_out ? reinterpret_cast<float4*>(P.st_out) + img * 2 * px : nullptr;
  J.x = P.x ? reinterpret_cast<float2*>(P.x) + img * px : nullptr;
  J.m = P.m;
  J.n = P.n;
  J.ty = t / P.tiles_x;
  J.tx = t - J.ty * P.tiles_x;
  J.lam = P.lam[img];
  J.c = P.c[img];
  J.R = P.R;
  J.T = P.T;
  J.r_hist = nullptr;
  J.hist_stride = 0;
  fgp_tile<KIND, CONSTR, MASK, RH>(J, P.halo, sBeta, sA1, sA2, sY);
}

// ---------------------------------------------------------------------------
// Batched kernel: one fused step (iterations k0+1 .. k0+T) for every image of a
// ragged batch. The tile list of the step holds, per image still running, the
// tiles laid out for that image's own halo (T_i + 1 when its last iteration
// falls in this step, else T_i), so each image is computed exactly as a plain
// call would. Each XCD owns one contiguous slice of the tile list and its
// workgroups stride through it; the plan launches one workgroup per tile (a
// persistent grid with static striding measured 15-20 % slower than letting
// the hardware dispatcher balance), so the loop normally runs once.
// ---------------------------------------------------------------------------
template <int CONSTR, int NW, int P>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void fgp_batched_kernel(FgpBatchedArgs A) {
  __shared__ float2 sBot[NW * kRW];
  __shared__ float2 sTop[NW * kRW];
  __shared__ float sBeta[kMaxFuse];
  if (threadIdx.x < kMaxFuse) sBeta[threadIdx.x] = (threadIdx.x < A.T) ? A.beta_table[A.k0 + 1 + threadIdx.x] : 0.0f;
  __syncthreads();
  constexpr int kXcd = 8;
  const int G = gridDim.x;
  const int xcd = blockIdx.x % kXcd, bi = blockIdx.x / kXcd;
  const int gx = G / kXcd + (xcd < G % kXcd ? 1 : 0);
  const int nrun = A.live ? A.live_count[0] : A.ntiles;
  const int lo = (int)((long long)nrun * xcd / kXcd);
  const int hi = (int)((long long)nrun * (xcd + 1) / kXcd);
  for (int t = lo + bi; t < hi; t += gx) {
    const BatchTile bt = A.tiles[A.live ? A.live[t] : t];
    const BatchImage D = A.images[bt.image];
    const int Ti = min(A.T, D.iters - A.k0);
    const bool last = (A.k0 + Ti == D.iters);
    const int H = max(1, Ti + (last ? 1 : 0));
    TileJob J;
    J.b = reinterpret_cast<const float2*>(A.b) + D.offset;
    J.mask = (D.support_offset >= 0 && A.support) ? A.support + D.support_offset : nullptr;
    J.st_in = (A.k0 == 0) ? nullptr : reinterpret_cast<const float4*>(A.st_in) + 2 * D.offset;
    J.st_out = last ? nullptr : reinterpret_cast<float4*>(A.st_out) + 2 * D.offset;
    J.x = last ? reinterpret_cast<float2*>(A.x) + D.offset : nullptr;
    J.m = D.m;
    J.n = D.n;
    J.tx = bt.tx;
    J.ty = bt.ty;
    J.lam = D.lam;
    J.c = D.c;
    J.R = D.R;
    J.T = Ti;
    J.r_hist = nullptr;
    J.hist_stride = 0;
    const int c0 = J.tx * (kRW - 2 * H) - H, r0 = J.ty * (NW * P - 2 * H) - H;
    const bool interior = c0 >= 1 && c0 + kRW <= J.n - 1 && r0 >= 1 && r0 + NW * P <= J.m - 1;
    const int sel = (D.kind * 2 + (J.mask ? 1 : 0)) * 2 + (interior ? 0 : 1);
    switch (sel) {
#define CTV_B(KI, MK, BO, S)                                                             \
  case S:                                                                                \
    fgp_tile_col<KI, CONSTR, MK, NW, P, BO>(J, H, sBeta, sBot, sTop);                    \
    break;
      CTV_B(K1I, false, false, 0) CTV_B(K1I, false, true, 1) CTV_B(K1I, true, false, 2) CTV_B(K1I, true, true, 3)
      CTV_B(K1A, false, false, 4) CTV_B(K1A, false, true, 5) CTV_B(K1A, true, false, 6) CTV_B(K1A, true, true, 7)
      CTV_B(K2I, false, false, 8) CTV_B(K2I, false, true, 9) CTV_B(K2I, true, false, 10) CTV_B(K2I, true, true, 11)
      CTV_B(K2A, false, false, 12) CTV_B(K2A, false, true, 13) CTV_B(K2A, true, false, 14)
      default: fgp_tile_col<K2A, CONSTR, true, NW, P, true>(J, H, sBeta, sBot, sTop); break;
#undef CTV_B
    }
    __syncthreads();  // the next tile reuses the LDS rows
  }
}

// ---------------------------------------------------------------------------
// Live tiles of a support (cold starts only). From q = 0 the dual stays exactly
// zero at a pixel outside the support whose lower and right neighbours are
// outside it too: y vanishes at all three pixels its differences read, so the
// gradient step adds nothing and P_S(0) = 0; x = 0 there as well. Such pixels
// are dead. A tile is live if its output holds a pixel that is not dead.
//
// live_scan_kernel: one workgroup of kScanWaves waves per tile of one image;
// lane = column of the output (plus one column to its right), each wave a
// band of the output rows. It writes flags[tile]; with zero_st it also stores
// zeros at the dead output pixels of both state buffers, for every image of
// the chunk (so tiles that later launches skip read and keep zeros); with x, a
// dead tile stores x = 0.
// ---------------------------------------------------------------------------
constexpr int kScanWaves = 4;

// Tile t of one image's tiling (halo, rows, tiles_x): returns whether it is
// live (the same value in every thread). st0 / st1 / x are image bases with
// `batch` images of stride 2 m n float4 / m n float2 (zeroed as described).
__device__ __forceinline__ bool scan_tile(const uint8_t* __restrict__ mask, int m, int n, int halo, int rows, int tiles_x, int t,
                          bool zero_st, float* st0, float* st1, float* x, int batch, int* sLive) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int OW = kRW - 2 * halo, OH = rows - 2 * halo;
  const int j0 = ty * OH, k = tx * OW + lane;
  const bool kin = lane <= OW && k < n;
  const bool kout = lane < OW && k < n;
  const long long px = (long long)m * n;
  const int jend = min(j0 + OH, m);  // output rows [j0, jend)
  const int band = (jend - j0 + kScanWaves - 1) / kScanWaves;
  const int jlo = j0 + wave * band, jhi = min(jend, jlo + band);
  bool below = (kin && jhi < m && jhi > jlo) ? (mask[(long long)jhi * n + k] != 0) : false;
  bool live = false;
  // Rows in chunks of kChunk, bottom up: every support byte of a chunk is
  // loaded before the first is tested (the zero stores in between would
  // otherwise order each load after the previous row's stores).
  constexpr int kChunk = 16;
  for (int top = jhi; top > jlo; top -= kChunk) {
    const int cnt = min(kChunk, top - jlo);  // rows top - 1, ..., top - cnt
    // unconditional loads from a clamped, valid position (a load in a branch of
    // its own waits for the one before it); the bytes that do not belong to
    // the band are zeroed afterwards
    const int kc = min(k, n - 1);
    int mb[kChunk];
#pragma unroll
    for (int i = 0; i < kChunk; ++i) mb[i] = mask[(long long)max(top - 1 - i, 0) * n + kc];
#pragma unroll
    for (int i = 0; i < kChunk; ++i) mb[i] = (kin && i < cnt) ? mb[i] : 0;
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
      if (i < cnt) {  // uniform over the wave
        const long long p = (long long)(top - 1 - i) * n + k;
        const bool cur = mb[i] != 0;
        const bool right = __shfl_down(cur ? 1 : 0, 1) != 0 && lane < 63;
        const bool dead = !cur && !below && !right;
        if (kout) {
          live = live || !dead;
          if (zero_st && dead) {
            const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int img = 0; img < batch; ++img) {
              const long long base = (long long)img * 2 * px;
              reinterpret_cast<float4*>(st0)[base + p] = z;
              reinterpret_cast<float4*>(st0)[base + px + p] = z;
              reinterpret_cast<float4*>(st1)[base + p] = z;
              reinterpret_cast<float4*>(st1)[base + px + p] = z;
            }
          }
        }
        below = cur;
      }
    }
  }
  const bool wave_live = __builtin_amdgcn_ballot_w64(live) != 0;
  if (lane == 0) sLive[wave] = wave_live ? 1 : 0;
  __syncthreads();
  bool tile_live = false;
  for (int w = 0; w < kScanWaves; ++w) tile_live = tile_live || sLive[w] != 0;
  if (!tile_live && x && kout) {
    for (int j = jlo; j < jhi; ++j)
      for (int img = 0; img < batch; ++img)
        reinterpret_cast<float2*>(x)[(long long)img * px + (long long)j * n + k] = make_float2(0.0f, 0.0f);
  }
  return tile_live;
}

__global__ __launch_bounds__(kScanWaves * 64) void live_scan_kernel(LiveScanArgs a) {
  __shared__ int sLive[kScanWaves];
  const bool live = scan_tile(a.mask, a.m, a.n, a.halo, a.rows, a.tiles_x, blockIdx.x, a.zero_st != 0, a.st0,
                              a.st1, a.x, a.batch, sLive);
  if (threadIdx.x == 0) a.flags[blockIdx.x] = live ? 1 : 0;
}

// Batched plans: one workgroup per tile of every (image, tiling) pair that the
// plan's steps use for images with a support (geo_of names the pair).
__global__ __launch_bounds__(kScanWaves * 64) void batched_scan_kernel(BatchScanArgs a) {
  __shared__ int sLive[kScanWaves];
  const int f = blockIdx.x;
  const BatchGeom G = a.geoms[a.geo_of[f]];
  const BatchImage D = a.images[G.image];
  const long long st = 2 * D.offset * 4;  // float offset of the image's state
  const int rows = a.sweep_oh > 0 ? a.sweep_oh + 2 * G.halo : a.rows;
  const bool live = scan_tile(a.support + D.support_offset, D.m, D.n, G.halo, rows, G.tiles_x,
                              f - G.flag_base, G.zero_st != 0, a.st0 + st, a.st1 + st,
                              G.zero_x ? a.x + 2 * D.offset : nullptr, 1, sLive);
  if (threadIdx.x == 0) a.flags[f] = live ? 1 : 0;
}

// Batched plans: one workgroup per step lists the step's tiles that run (tiles
// of images without a support always run; the others by their flag), in
// order, at lists[step_offset] with the count in counts[step].
__global__ __launch_bounds__(1024) void batched_compact_kernel(BatchCompactArgs a) {
  __shared__ int sWave[16];
  const int s = blockIdx.x;
  const BatchTile* tiles = a.tiles + a.step_offset[s];
  const int count = a.step_count[s];
  int* list = a.lists + a.step_offset[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (count + 1023) / 1024;
  const int lo = min(count, tid * per), hi = min(count, lo + per);
  int own = 0;
  for (int i = lo; i < hi; ++i) own += (tiles[i].flag < 0 || a.flags[tiles[i].flag] != 0) ? 1 : 0;
  int inc = own;
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) sWave[wave] = inc;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < 16; ++w) {
    const int v = sWave[w];
    before += (w < wave) ? v : 0;
    total += v;
  }
  if (tid == 0) a.counts[s] = total;
  int pos = before + inc - own;
  for (int i = lo; i < hi; ++i)
    if (tiles[i].flag < 0 || a.flags[tiles[i].flag] != 0) list[pos++] = i;
}

const void* batched_scan_kernel_ptr() { return reinterpret_cast<const void*>(&batched_scan_kernel); }
const void* batched_compact_kernel_ptr() { return reinterpret_cast<const void*>(&batched_compact_kernel); }

// One workgroup: live[0] = number of live tiles, live[1 ..] = their indices in
// increasing order (each thread takes a contiguous run of flags; a block-wide
// exclusive scan of the run counts places the runs).
__global__ __launch_bounds__(1024) void live_list_kernel(const int* __restrict__ flags, int count,
                                                          int* __restrict__ live) {
  __shared__ int sWave[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (count + 1023) / 1024;
  const int lo = min(count, tid * per), hi = min(count, lo + per);
  int own = 0;
  for (int i = lo; i < hi; ++i) own += flags[i] != 0;
  int inc = own;
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) sWave[wave] = inc;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < 16; ++w) {
    const int v = sWave[w];
    before += (w < wave) ? v : 0;
    total += v;
  }
  if (tid == 0) live[0] = total;
  int pos = 1 + before + inc - own;
  for (int i = lo; i < hi; ++i)
    if (flags[i] != 0) live[pos++] = i;
}

hipError_t launch_live_tiles(const LiveScanArgs& a, int* live, hipStream_t s) {
  const int count = a.tiles_x * a.tiles_y;
  if (a.halo < 1 || kRW - 2 * a.halo < 1 || a.rows - 2 * a.halo < 1 || count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(live_scan_kernel, dim3(count), dim3(kScanWaves * 64), 0, s, a);
  hipLaunchKernelGGL(live_list_kernel, dim3(1), dim3(1024), 0, s, a.flags, count, live);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Zero fill (used instead of a memset node so calls stay safe to capture).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void zero_f4_kernel(float4* __restrict__ p, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

hipError_t launch_zero_f4(float* p, long long count_f4, hipStream_t s) {
  if (count_f4 <= 0) return hipSuccess;
  const int nb = (int)((count_f4 + 255) / 256);
  hipLaunchKernelGGL(zero_f4_kernel, dim3(nb), dim3(256), 0, s, reinterpret_cast<float4*>(p), count_f4);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// x = P_C(b) (lambda = 0 or K = 0).
// ---------------------------------------------------------------------------
template <int CONSTR>
__global__ __launch_bounds__(256) void project_c_kernel(const float2* __restrict__ b,
                                                        const uint8_t* __restrict__ mask,
                                                        float2* __restrict__ x, long long px,
                                                        long long total) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const bool in = mask ? (mask[i % px] != 0) : true;
  x[i] = proj_c<CONSTR>(b[i], in);
}

// ---------------------------------------------------------------------------
// Duality gap: per pixel the group term(s)
//   ||(L x)_g||_* - <q_g, (L x)_g>  (weighted by alpha / 1-alpha for type-II),
// nonnegative for q in S; reduced in float64, deterministically.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ double gap_term(float4 q, float2 x, float2 xd, float2 xr, bool hd,
                                           bool hr, const Radii& R) {
  const float u1 = hd ? x.x - xd.x : 0.0f, v1 = hd ? x.y - xd.y : 0.0f;
  const float u2 = hr ? x.x - xr.x : 0.0f, v2 = hr ? x.y - xr.y : 0.0f;
  const double dot = (double)q.x * u1 + (double)q.y * v1 + (double)q.z * u2 + (double)q.w * v2;
  double nrm;
  if (KIND == K1I) {
    nrm = sqrt((double)u1 * u1 + (double)v1 * v1 + (double)u2 * u2 + (double)v2 * v2);
  } else if (KIND == K1A) {
    nrm = sqrt((double)u1 * u1 + (double)v1 * v1) + sqrt((double)u2 * u2 + (double)v2 * v2);
  } else if (KIND == K2I) {
    nrm = (double)R.ra * sqrt((double)u1 * u1 + (double)u2 * u2) +
          (double)R.sa * sqrt((double)v1 * v1 + (double)v2 * v2);
  } else {
    nrm = (double)R.ra * (fabs((double)u1) + fabs((double)u2)) +
          (double)R.sa * (fabs((double)v1) + fabs((double)v2));
  }
  return nrm - dot;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
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

template <int KIND>
__global__ __launch_bounds__(256) void gap_partial_kernel(const float2* __restrict__ x,
                                                          const float4* __restrict__ st,
                                                          int m, int n, Radii R, int blocks_per_img,
                                                          double* __restrict__ partial) {
  __shared__ double red[4];
  const int img = blockIdx.x / blocks_per_img;
  const int blk = blockIdx.x - img * blocks_per_img;
  const long long px = (long long)m * n;
  const float2* xi = x + img * px;
  const float4* qi = st + img * 2 * px;
  double acc = 0.0;
  for (long long p = (long long)blk * blockDim.x + threadIdx.x; p < px;
       p += (long long)blocks_per_img * blockDim.x) {
    const int j = (int)(p / n), k = (int)(p - (long long)j * n);
    const bool hd = j < m - 1, hr = k < n - 1;
    const float2 xv = xi[p];
    const float2 xd = hd ? xi[p + n] : xv;
    const float2 xr = hr ? xi[p + 1] : xv;
    acc += gap_term<KIND>(qi[p], xv, xd, xr, hd, hr, R);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// One wave per image: lane l adds the blocks l, l + 64, ... in order, then a
// fixed butterfly combines the lanes (the same summation order on every run).
__global__ __launch_bounds__(64) void gap_final_kernel(const double* __restrict__ partial, int blocks_per_img,
                                                       GapArgs L, double* __restrict__ gap, int batch) {
  const int img = blockIdx.x;
  double s = 0.0;
  for (int i = (int)threadIdx.x; i < blocks_per_img; i += 64) s += partial[img * blocks_per_img + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0 && img < batch) gap[img] = (double)L.lam[img] * s;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <int KIND, int CONSTR, bool MASK>
static hipError_t launch_plain_rh(const FgpPlainArgs& a, int rh, int nblocks, hipStream_t s) {
  if (rh == 32)
    hipLaunchKernelGGL((fgp_plain_kernel<KIND, CONSTR, MASK, 32>), dim3(nblocks), dim3(kThreads), 0, s, a);
  else if (rh == 64)
    hipLaunchKernelGGL((fgp_plain_kernel<KIND, CONSTR, MASK, 64>), dim3(nblocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((fgp_plain_kernel<KIND, CONSTR, MASK, 16>), dim3(nblocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_plain_kind(const FgpPlainArgs& a, int constr, bool mask, int rh, int nb,
                                    hipStream_t s) {
  if (constr == C_MOD)
    return mask ? launch_plain_rh<KIND, C_MOD, true>(a, rh, nb, s)
                : launch_plain_rh<KIND, C_MOD, false>(a, rh, nb, s);
  return mask ? launch_plain_rh<KIND, C_NONE, true>(a, rh, nb, s)
              : launch_plain_rh<KIND, C_NONE, false>(a, rh, nb, s);
}

template <int KIND, int CONSTR, bool MASK>
static hipError_t launch_col_shape(const FgpPlainArgs& a, int nw, int p, int nb, hipStream_t s) {
  if (a.r_hist) {   // the r-history variant exists for the default 8 x 8 shape only
    if (nw != 8 || p != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((fgp_col_kernel<KIND, CONSTR, MASK, 8, 8, true>), dim3(nb), dim3(8 * 64), 0, s, a);
    return hipGetLastError();
  }
#define CTV_COL(NW_, P_)                                                                        \
  if (nw == NW_ && p == P_) {                                                                   \
    hipLaunchKernelGGL((fgp_col_kernel<KIND, CONSTR, MASK, NW_, P_>), dim3(nb), dim3(NW_ * 64), 0, s, a); \
    return hipGetLastError();                                                                   \
  }
  CTV_COL(4, 8)
  CTV_COL(8, 4)
  CTV_COL(8, 8)
  CTV_COL(12, 4)
  CTV_COL(16, 4)
  CTV_COL(16, 8)
#undef CTV_COL
  return hipErrorInvalidValue;
}

template <int KIND>
static hipError_t launch_col_kind(const FgpPlainArgs& a, int constr, bool mask, int nw, int p, int nb,
                                  hipStream_t s) {
  if (constr == C_MOD)
    return mask ? launch_col_shape<KIND, C_MOD, true>(a, nw, p, nb, s)
                : launch_col_shape<KIND, C_MOD, false>(a, nw, p, nb, s);
  return mask ? launch_col_shape<KIND, C_NONE, true>(a, nw, p, nb, s)
              : launch_col_shape<KIND, C_NONE, false>(a, nw, p, nb, s);
}

hipError_t launch_fgp_plain(const FgpPlainArgs& a, int kind, int constr, const TileShape& ts, int batch,
                            hipStream_t s) {
  if (ts.sweep()) return launch_fgp_sweep(a, kind, constr, batch, s);
  const int nblocks = a.tiles_x * a.tiles_y * batch;
  const bool mask = a.mask != nullptr;
  if (ts.waves > 0) {
    switch (kind) {
      case K1I: return launch_col_kind<K1I>(a, constr, mask, ts.waves, ts.rows_per_thread, nblocks, s);
      case K1A: return launch_col_kind<K1A>(a, constr, mask, ts.waves, ts.rows_per_thread, nblocks, s);
      case K2I: return launch_col_kind<K2I>(a, constr, mask, ts.waves, ts.rows_per_thread, nblocks, s);
      default: return launch_col_kind<K2A>(a, constr, mask, ts.waves, ts.rows_per_thread, nblocks, s);
    }
  }
  const int rh = ts.rows_per_thread * kWaves;
  switch (kind) {
    case K1I: return launch_plain_kind<K1I>(a, constr, mask, rh, nblocks, s);
    case K1A: return launch_plain_kind<K1A>(a, constr, mask, rh, nblocks, s);
    case K2I: return launch_plain_kind<K2I>(a, constr, mask, rh, nblocks, s);
    default: return launch_plain_kind<K2A>(a, constr, mask, rh, nblocks, s);
  }
}

template <int KIND>
static const void* flow_kernel_ptr(int constr, bool mask) {
  if (constr == C_MOD)
    return mask ? reinterpret_cast<const void*>(&fgp_flow_kernel<KIND, C_MOD, true>)
                : reinterpret_cast<const void*>(&fgp_flow_kernel<KIND, C_MOD, false>);
  return mask ? reinterpret_cast<const void*>(&fgp_flow_kernel<KIND, C_NONE, true>)
              : reinterpret_cast<const void*>(&fgp_flow_kernel<KIND, C_NONE, false>);
}

template <int KIND>
static hipError_t launch_single_kind(const FgpSingleArgs& a, int constr, int batch, hipStream_t s) {
  const bool mask = a.mask != nullptr;
  if (constr == C_MOD) {
    if (mask) hipLaunchKernelGGL((fgp_single_kernel<KIND, C_MOD, true>), dim3(batch), dim3(kSingleNW * 64), 0, s, a);
    else hipLaunchKernelGGL((fgp_single_kernel<KIND, C_MOD, false>), dim3(batch), dim3(kSingleNW * 64), 0, s, a);
  } else {
    if (mask) hipLaunchKernelGGL((fgp_single_kernel<KIND, C_NONE, true>), dim3(batch), dim3(kSingleNW * 64), 0, s, a);
    else hipLaunchKernelGGL((fgp_single_kernel<KIND, C_NONE, false>), dim3(batch), dim3(kSingleNW * 64), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fgp_single(const FgpSingleArgs& a, int kind, int constr, int batch, hipStream_t s) {
  if (a.m > kSingleNW * kSingleP || a.n > kRW || a.T < 0 || a.T > kFlowMaxIters) return hipErrorInvalidValue;
  switch (kind) {
    case K1I: return launch_single_kind<K1I>(a, constr, batch, s);
    case K1A: return launch_single_kind<K1A>(a, constr, batch, s);
    case K2I: return launch_single_kind<K2I>(a, constr, batch, s);
    default: return launch_single_kind<K2A>(a, constr, batch, s);
  }
}

long long flow_ints(int batch, int m, int n, int h) {
  const long long tx = (n + (kRW - 2 * h) - 1) / (kRW - 2 * h);
  const long long ty = (m + (64 - 2 * h) - 1) / (64 - 2 * h);
  return 64 + (long long)batch * tx * ty;
}

hipError_t launch_fgp_flow(const FgpFlowArgs& a, int kind, int constr, hipStream_t s) {
  const bool mask = a.mask != nullptr;
  const void* fn = nullptr;
  switch (kind) {
    case K1I: fn = flow_kernel_ptr<K1I>(constr, mask); break;
    case K1A: fn = flow_kernel_ptr<K1A>(constr, mask); break;
    case K2I: fn = flow_kernel_ptr<K2I>(constr, mask); break;
    default: fn = flow_kernel_ptr<K2A>(constr, mask); break;
  }
  // One workgroup per resident slot: a ticket is only taken by a running
  // workgroup, and every task waits only on tasks with smaller tickets.
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 512, 0);
  if (e != hipSuccess) return e;
  const long long total = (long long)a.tiles_x * a.tiles_y * a.batch * (a.steps + 1);
  const int grid = (int)std::max(1LL, std::min<long long>((long long)std::max(per_cu, 1) * cus, total));
  void* args[] = {const_cast<FgpFlowArgs*>(&a)};
  return hipLaunchKernel(fn, dim3(grid), dim3(512), args, 0, s);
}

const void* fgp_batched_kernel_ptr(int constr, const TileShape& ts) {
  if (ts.sweep()) return fgp_sweep_batched_kernel_ptr(constr);
#define CTV_BK(NW_, P_)                                                                      \
  if (ts.waves == NW_ && ts.rows_per_thread == P_)                                           \
    return constr == C_MOD ? reinterpret_cast<const void*>(&fgp_batched_kernel<C_MOD, NW_, P_>) \
                           : reinterpret_cast<const void*>(&fgp_batched_kernel<C_NONE, NW_, P_>);
  CTV_BK(8, 8)
  CTV_BK(8, 4)
  CTV_BK(12, 4)
  CTV_BK(16, 4)
#undef CTV_BK
  return nullptr;
}

hipError_t launch_project_c(const float* b, const uint8_t* mask, float* x, long long px,
                            int batch, int constr, hipStream_t s) {
  const long long total = px * batch;
  const int nb = (int)((total + 255) / 256);
  if (constr == C_MOD)
    hipLaunchKernelGGL(project_c_kernel<C_MOD>, dim3(nb), dim3(256), 0, s,
                       reinterpret_cast<const float2*>(b), mask, reinterpret_cast<float2*>(x), px, total);
  else
    hipLaunchKernelGGL(project_c_kernel<C_NONE>, dim3(nb), dim3(256), 0, s,
                       reinterpret_cast<const float2*>(b), mask, reinterpret_cast<float2*>(x), px, total);
  return hipGetLastError();
}

hipError_t launch_gap(const float* x, const float* state, int m, int n, int batch, int kind,
                      Radii R, const GapArgs& lam, double* partial, int blocks_per_img,
                      double* gap, hipStream_t s) {
  const float2* xx = reinterpret_cast<const float2*>(x);
  const float4* st = reinterpret_cast<const float4*>(state);
  const int nb = blocks_per_img * batch;
  switch (kind) {
    case K1I: hipLaunchKernelGGL(gap_partial_kernel<K1I>, dim3(nb), dim3(256), 0, s, xx, st, m, n, R, blocks_per_img, partial); break;
    case K1A: hipLaunchKernelGGL(gap_partial_kernel<K1A>, dim3(nb), dim3(256), 0, s, xx, st, m, n, R, blocks_per_img, partial); break;
    case K2I: hipLaunchKernelGGL(gap_partial_kernel<K2I>, dim3(nb), dim3(256), 0, s, xx, st, m, n, R, blocks_per_img, partial); break;
    default: hipLaunchKernelGGL(gap_partial_kernel<K2A>, dim3(nb), dim3(256), 0, s, xx, st, m, n, R, blocks_per_img, partial); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gap_final_kernel, dim3((unsigned)batch), dim3(64), 0, s, partial, blocks_per_img, lam,
                     gap, batch);
  return hipGetLastError();
}

}  // namespace ctv
