// Row-sweep tile of the fused FGP iteration (Algorithm 2, lines 3-5, T
// iterations per launch): a workgroup owns a strip of 64 columns and a segment
// of SH output rows, and sweeps down the segment in bands of 32 rows without
// recomputing any row above or below a band.
//
// Skew. One iteration at row j reads the previous iterate at rows j-1, j and
// j+1 only. So a wave whose window at iteration (level) t covers rows
// [a - t, a + P - t) - one row higher per level - has everything it needs in
// its own registers except the new top row, which the wave above (or, for the
// top wave, the previous band's bottom wave) computed at level t-1 and hands
// over. Each level a wave gives away its bottom row (level t-1 state q, r and
// y = P_C(b - lambda L^T r) of level t, which it needs itself for its own
// bottom row's gradient step) and receives a new top row, through LDS: one
// barrier per level, no vertical halo inside the segment. The window is a
// circular buffer of P register slots (row j lives in slot j mod P), so the
// hand-over moves no registers: level t's code is specialised on t mod P.
//
// Segment edges. The loaded rows of a segment with output rows [j0, j1) are
// [j0 - T - e, j1 + T) (e = 1 when the launch writes x, whose Eq. (18) reads
// q one row up); at level t only rows [j0 - e - (T - t), j1 + (T - t)) can
// still reach the output, and bands that reach outside it, or the image
// border, run a variant with per-row guards. Columns keep the halo of the
// column-register tile (64 - 2H output columns, H = T + e).
//
// Every pixel runs the shared per-pixel operators (ctv_device.hpp), so results
// are bitwise those of every other tile kernel.
#include <hip/hip_runtime.h>

#include "ctv_device.hpp"
#include "ctv_kernels.hpp"
#include "ctv_tile.hpp"

namespace ctv {

namespace {

constexpr int NW = kSweepWaves;   // waves per workgroup
constexpr int P = kSweepRows;     // rows per wave window
constexpr int RB = NW * P;        // rows per band
constexpr int RING = kSweepMaxFuse + 2;

// LDS: the level-to-level hand-over between the waves of a band (double
// buffered by level parity), the ring that carries the bottom wave's rows to
// the next band's top wave (written at level g, read at level g + T; a ring
// of T + 2 slots keeps every slot alive until it is read), and the q rows the
// Eq. (18) epilogue needs from the wave above.
struct SweepLds {
  float4 lq[2][NW - 1][kRW];
  float4 lr[2][NW - 1][kRW];
  float2 ly[2][NW - 1][kRW];
  float4 cq[RING][kRW];
  float4 cr[RING][kRW];
  float2 cy[RING][kRW];
  float2 up[NW][kRW];
  float beta[kMaxFuse];
};

// Uniform state of one wave in one segment.
struct Sweep {
  int lane, wave;
  int k;                 // this lane's column
  bool kin, has_left, has_right, col_out;
  int m, n, T, e;
  int j0, j1;            // output rows of the segment
  int A0;                // first loaded row: j0 - T - e
  float lam, c;
  Radii R;
  long long plane;
};

struct Window {
  float4 q[P], r[P];
  float2 b[P];
  int in[P];             // the support byte (nonzero = inside), kept raw so that a load of it is
                         // waited for only where it is used
  float2 xup;            // wave 0: q (r1, s1) of the previous band's last row, for Eq. (18)
};

// Barrier for the LDS hand-over only: global loads issued before it stay in
// flight (the rows' b and support for later levels).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// b, support byte and (with_state) the dual state of row j for this lane's
// column. EDGE: zeros outside the image; otherwise the row and column are
// known to lie inside and the loads are unconditional.
template <bool MASK, bool EDGE>
__device__ __forceinline__ void load_row(const TileJob& J, const Sweep& S, int j, bool with_state, float4& q,
                                         float4& r, float2& b, int& in) {
  if (!EDGE) {
    const long long p = (long long)j * S.n + S.k;
    b = J.b[p];
    in = MASK ? (int)J.mask[p] : 1;
    if (with_state) {
      q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      r = q;
      if (J.st_in) {
        q = J.st_in[p];
        r = J.st_in[S.plane + p];
      }
    }
    return;
  }
  b = make_float2(0.0f, 0.0f);
  in = MASK ? 0 : 1;
  if (with_state) {
    q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    r = q;
  }
  if (S.kin && j >= 0 && j < S.m) {
    const long long p = (long long)j * S.n + S.k;
    b = J.b[p];
    if (MASK) in = J.mask[p];
    if (with_state && J.st_in) {
      q = J.st_in[p];
      r = J.st_in[S.plane + p];
    }
  }
}

// One level t (t mod P = PHI) of one wave. EDGE: per-row guards for rows that
// cannot reach the output or lie on / outside the image border.
template <int KIND, int CONSTR, bool MASK, bool EDGE, int PHI>
__device__ __forceinline__ void sweep_level(const TileJob& J, const Sweep& S, Window& W, SweepLds& L, int a, int t,
                                            int g) {
  constexpr int TOP = (P - PHI) % P;   // slot of the leaving row (level t-1) = slot of the entering row
  constexpr int PRE = (TOP + P - 1) % P;
  const float2 zero2 = make_float2(0.0f, 0.0f);
  const int e = a - t;                 // entering (top) row of the level-t window; the leaving row is e + P
  // rows that can still reach the output at this level: q on [lo, hi), y on [lo, hi]
  const int lo = max(S.A0 + t, 0);
  const int hi = min(S.j1 + S.T - t, S.m);

  // (a) y of the leaving row at level t, from level t-1 values this wave holds
  const int jl = e + P;
  float2 yl = zero2;
  if (!EDGE || (jl >= lo && jl <= hi && jl < S.m)) {
    float2 up = make_float2(W.r[PRE].x, W.r[PRE].y);
    float2 left = make_float2(lane_from_left(W.r[TOP].z), lane_from_left(W.r[TOP].w));
    if (EDGE) {
      up = (jl > 0) ? up : zero2;
      left = S.has_left ? left : zero2;
    }
    yl = proj_c<CONSTR>(dual_to_primal(W.b[TOP], W.r[TOP], up, left, S.lam), W.in[TOP] != 0);
  }
  const int par = t & 1;
  if (S.wave < NW - 1) {
    L.lq[par][S.wave][S.lane] = W.q[TOP];
    L.lr[par][S.wave][S.lane] = W.r[TOP];
    L.ly[par][S.wave][S.lane] = yl;
  } else {
    const int slot = g % RING;
    L.cq[slot][S.lane] = W.q[TOP];
    L.cr[slot][S.lane] = W.r[TOP];
    L.cy[slot][S.lane] = yl;
  }
  lds_barrier();
  // (b) the entering row (level t-1 state and its level-t y) replaces the leaving one
  float2 y[P + 1];
  if (S.wave > 0) {
    W.q[TOP] = L.lq[par][S.wave - 1][S.lane];
    W.r[TOP] = L.lr[par][S.wave - 1][S.lane];
    y[0] = L.ly[par][S.wave - 1][S.lane];
  } else {
    const int slot = ((g - S.T) % RING + RING) % RING;
    W.q[TOP] = L.cq[slot][S.lane];
    W.r[TOP] = L.cr[slot][S.lane];
    y[0] = L.cy[slot][S.lane];
  }
  y[P] = yl;
  {
    float4 dq, dr;
    load_row<MASK, EDGE>(J, S, e, false, dq, dr, W.b[TOP], W.in[TOP]);   // first used at the next level
  }
  // (c) y of the other window rows
#pragma unroll
  for (int i = 1; i < P; ++i) {
    const int s = (TOP + i) % P, sp = (TOP + i - 1) % P;
    const int j = e + i;
    if (!EDGE || (j >= lo && j <= hi && j < S.m)) {
      float2 up = make_float2(W.r[sp].x, W.r[sp].y);
      float2 left = make_float2(lane_from_left(W.r[s].z), lane_from_left(W.r[s].w));
      if (EDGE) {
        up = (j > 0) ? up : zero2;
        left = S.has_left ? left : zero2;
      }
      y[i] = proj_c<CONSTR>(dual_to_primal(W.b[s], W.r[s], up, left, S.lam), W.in[s] != 0);
    } else {
      y[i] = zero2;
    }
  }
  // (d) gradient step and dual update of the window rows
  const float beta = L.beta[t - 1];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int s = (TOP + i) % P;
    const int j = e + i;
    if (!EDGE || (j >= lo && j < hi)) {
      const float rx = lane_from_right(y[i].x), ry = lane_from_right(y[i].y);
      const float4 gv = dual_step(W.r[s], y[i], y[i + 1], make_float2(rx, ry), S.c, !EDGE || j < S.m - 1,
                                  !EDGE || S.has_right);
      dual_update<KIND>(gv, S.R, beta, W.q[s], W.r[s]);
    }
  }
}

// After the last level: store the state of the output rows and, with x, the
// Eq. (18) output. The window's row i (from the top) is a - T + i in slot
// (i - T) mod P, i.e. (TOPT + i) mod P.
template <int CONSTR, bool EDGE, int TOPT>
__device__ __forceinline__ void sweep_finish(const TileJob& J, const Sweep& S, Window& W, SweepLds& L, int a) {
  const float2 zero2 = make_float2(0.0f, 0.0f);
  const int top = a - S.T;
  if (J.x) {
    constexpr int BOT = (TOPT + P - 1) % P;
    L.up[S.wave][S.lane] = make_float2(W.q[BOT].x, W.q[BOT].y);
    lds_barrier();
    float2 up0 = W.xup;
    if (S.wave > 0) {
      up0 = L.up[S.wave - 1][S.lane];
    } else {
      W.xup = L.up[NW - 1][S.lane];   // for the next band
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int s = (TOPT + i) % P, sp = (TOPT + i + P - 1) % P;
      const int j = top + i;
      if (j >= S.j0 && j < S.j1) {
        float2 up = (i > 0) ? make_float2(W.q[sp].x, W.q[sp].y) : up0;
        float2 left = make_float2(lane_from_left(W.q[s].z), lane_from_left(W.q[s].w));
        if (EDGE) {
          up = (j > 0) ? up : zero2;
          left = S.has_left ? left : zero2;
        }
        const float2 xv = proj_c<CONSTR>(dual_to_primal(W.b[s], W.q[s], up, left, S.lam), W.in[s] != 0);
        if (S.col_out) store_nt(J.x + (long long)j * S.n + S.k, xv);
      }
    }
  }
  if (J.st_out) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int s = (TOPT + i) % P;
      const int j = top + i;
      if (j >= S.j0 && j < S.j1 && S.col_out) {
        const long long p = (long long)j * S.n + S.k;
        store_nt(J.st_out + p, W.q[s]);
        store_nt(J.st_out + S.plane + p, W.r[s]);
      }
    }
  }
}

// Level t (phase PHI = t mod P), and after the last level the band's outputs.
template <int KIND, int CONSTR, bool MASK, bool EDGE, int PHI>
__device__ __forceinline__ void sweep_step(const TileJob& J, const Sweep& S, Window& W, SweepLds& L, int a, int t,
                                           int s) {
  sweep_level<KIND, CONSTR, MASK, EDGE, PHI>(J, S, W, L, a, t, s * S.T + t);
  if (t == S.T) sweep_finish<CONSTR, EDGE, (P - PHI) % P>(J, S, W, L, a);
}

// One band: load the level-0 rows, run the levels (written out in phase
// order, so that every register slot index is a compile-time constant), store.
template <int KIND, int CONSTR, bool MASK, bool EDGE>
__device__ __forceinline__ void sweep_band(const TileJob& J, const Sweep& S, Window& W, SweepLds& L, int A, int s) {
  const int a = A + S.wave * P;
#pragma unroll
  for (int i = 0; i < P; ++i) load_row<MASK, EDGE>(J, S, a + i, true, W.q[i], W.r[i], W.b[i], W.in[i]);
  if (S.T == 0) sweep_finish<CONSTR, EDGE, 0>(J, S, W, L, a);   // no iterations (lambda = 0 or K = 0): Eq. (18) only
  for (int t = 1; t <= S.T; t += P) {
    sweep_step<KIND, CONSTR, MASK, EDGE, 1>(J, S, W, L, a, t, s);
    if (t + 1 <= S.T) sweep_step<KIND, CONSTR, MASK, EDGE, 2>(J, S, W, L, a, t + 1, s);
    if (t + 2 <= S.T) sweep_step<KIND, CONSTR, MASK, EDGE, 3>(J, S, W, L, a, t + 2, s);
    if (t + 3 <= S.T) sweep_step<KIND, CONSTR, MASK, EDGE, 0>(J, S, W, L, a, t + 3, s);
  }
}

// One tile: strip J.tx (64 - 2H output columns), segment J.ty (SH output rows).
template <int KIND, int CONSTR, bool MASK>
__device__ __forceinline__ void fgp_tile_sweep(const TileJob& J, int H, int SH, SweepLds& L) {
  static_assert(P == 4, "the level and finish switches assume four rows per wave");
  Sweep S;
  S.lane = threadIdx.x & 63;
  S.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  S.m = J.m;
  S.n = J.n;
  S.T = J.T;
  S.e = J.x ? 1 : 0;
  const int OW = kRW - 2 * H;
  const int c0 = J.tx * OW - H;
  S.k = c0 + S.lane;
  S.kin = S.k >= 0 && S.k < J.n;
  S.has_left = S.k > 0;
  S.has_right = S.k < J.n - 1;
  S.col_out = S.lane >= H && S.lane < kRW - H && S.kin;
  S.j0 = J.ty * SH;
  S.j1 = min(S.j0 + SH, J.m);
  S.A0 = S.j0 - S.T - S.e;
  S.lam = J.lam;
  S.c = J.c;
  S.R = J.R;
  S.plane = (long long)J.m * J.n;
  const bool strip_inside = c0 >= 1 && c0 + kRW <= J.n - 1;
  Window W;
  W.xup = make_float2(0.0f, 0.0f);
  for (int s = 0;; ++s) {
    const int A = S.A0 + s * RB;
    if (A - S.T >= S.j1) break;
    // a band runs without guards when every row it touches is inside the image
    // (not on its border) and every row of its windows can reach the output
    const bool clean = strip_inside && A - S.T >= S.j0 - S.e && A + RB <= S.j1 + S.T && A - S.T >= 1 &&
                       A + RB <= S.m - 1;
    if (clean)
      sweep_band<KIND, CONSTR, MASK, false>(J, S, W, L, A, s);
    else
      sweep_band<KIND, CONSTR, MASK, true>(J, S, W, L, A, s);
  }
}

}  // namespace

// Plain launch: one workgroup per tile of the chunk (tiles_x strips x tiles_y
// segments per image), or per entry of the live-tile list.
template <int KIND, int CONSTR, bool MASK>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void fgp_sweep_kernel(FgpPlainArgs A_) {
  __shared__ SweepLds L;
  if (threadIdx.x < kMaxFuse) L.beta[threadIdx.x] = A_.beta[threadIdx.x];
  __syncthreads();
  const int per_img = A_.tiles_x * A_.tiles_y;
  int img, t;
  if (A_.live) {
    const int Lc = A_.live[0];
    const int total = (gridDim.x / per_img) * Lc;
    constexpr int kXcd = 8;
    const int x = blockIdx.x % kXcd, i = blockIdx.x / kXcd;
    const int q = total / kXcd, rem = total % kXcd;
    if (i >= q + (x < rem ? 1 : 0)) return;
    const int en = x * q + (x < rem ? x : rem) + i;
    img = en / Lc;
    t = A_.live[1 + (en - img * Lc)];
  } else {
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    img = tile / per_img;
    t = tile - img * per_img;
  }
  const long long px = (long long)A_.m * A_.n;
  TileJob J;
  J.b = reinterpret_cast<const float2*>(A_.b) + img * px;
  J.mask = A_.mask;
  J.st_in = A_.st_in ? reinterpret_cast<const float4*>(A_.st_in) + img * 2 * px : nullptr;
  J.st_out = A_.st_out ? reinterpret_cast<float4*>(A_.st_out) + img * 2 * px : nullptr;
  J.x = A_.x ? reinterpret_cast<float2*>(A_.x) + img * px : nullptr;
  J.m = A_.m;
  J.n = A_.n;
  J.ty = t / A_.tiles_x;
  J.tx = t - J.ty * A_.tiles_x;
  J.lam = A_.lam[img];
  J.c = A_.c[img];
  J.R = A_.R;
  J.T = A_.T;
  J.r_hist = nullptr;
  J.hist_stride = 0;
  fgp_tile_sweep<KIND, CONSTR, MASK>(J, A_.halo, A_.sweep_rows, L);
}

// Batched launch: one fused step of a ragged batch (see fgp_batched_kernel);
// each tile is a (strip, segment) of its image at the image's own halo.
template <int CONSTR>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void fgp_sweep_batched_kernel(
    FgpBatchedArgs A_) {
  __shared__ SweepLds L;
  if (threadIdx.x < kMaxFuse)
    L.beta[threadIdx.x] = (threadIdx.x < A_.T) ? A_.beta_table[A_.k0 + 1 + threadIdx.x] : 0.0f;
  __syncthreads();
  constexpr int kXcd = 8;
  const int G = gridDim.x;
  const int xcd = blockIdx.x % kXcd, bi = blockIdx.x / kXcd;
  const int gx = G / kXcd + (xcd < G % kXcd ? 1 : 0);
  const int nrun = A_.live ? A_.live_count[0] : A_.ntiles;
  const int lo = (int)((long long)nrun * xcd / kXcd);
  const int hi = (int)((long long)nrun * (xcd + 1) / kXcd);
  for (int t = lo + bi; t < hi; t += gx) {
    const BatchTile bt = A_.tiles[A_.live ? A_.live[t] : t];
    const BatchImage D = A_.images[bt.image];
    const int Ti = min(A_.T, D.iters - A_.k0);
    const bool last = (A_.k0 + Ti == D.iters);
    const int H = max(1, Ti + (last ? 1 : 0));
    TileJob J;
    J.b = reinterpret_cast<const float2*>(A_.b) + D.offset;
    J.mask = (D.support_offset >= 0 && A_.support) ? A_.support + D.support_offset : nullptr;
    J.st_in = (A_.k0 == 0) ? nullptr : reinterpret_cast<const float4*>(A_.st_in) + 2 * D.offset;
    J.st_out = last ? nullptr : reinterpret_cast<float4*>(A_.st_out) + 2 * D.offset;
    J.x = last ? reinterpret_cast<float2*>(A_.x) + D.offset : nullptr;
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
    const int sel = D.kind * 2 + (J.mask ? 1 : 0);
    switch (sel) {
      case 0: fgp_tile_sweep<K1I, CONSTR, false>(J, H, A_.sweep_rows, L); break;
      case 1: fgp_tile_sweep<K1I, CONSTR, true>(J, H, A_.sweep_rows, L); break;
      case 2: fgp_tile_sweep<K1A, CONSTR, false>(J, H, A_.sweep_rows, L); break;
      case 3: fgp_tile_sweep<K1A, CONSTR, true>(J, H, A_.sweep_rows, L); break;
      case 4: fgp_tile_sweep<K2I, CONSTR, false>(J, H, A_.sweep_rows, L); break;
      case 5: fgp_tile_sweep<K2I, CONSTR, true>(J, H, A_.sweep_rows, L); break;
      case 6: fgp_tile_sweep<K2A, CONSTR, false>(J, H, A_.sweep_rows, L); break;
      default: fgp_tile_sweep<K2A, CONSTR, true>(J, H, A_.sweep_rows, L); break;
    }
    __syncthreads();  // the next tile reuses the LDS
  }
}

template <int KIND>
static hipError_t launch_sweep_kind(const FgpPlainArgs& a, int constr, bool mask, int nblocks, hipStream_t s) {
  if (constr == C_MOD) {
    if (mask) hipLaunchKernelGGL((fgp_sweep_kernel<KIND, C_MOD, true>), dim3(nblocks), dim3(NW * 64), 0, s, a);
    else hipLaunchKernelGGL((fgp_sweep_kernel<KIND, C_MOD, false>), dim3(nblocks), dim3(NW * 64), 0, s, a);
  } else {
    if (mask) hipLaunchKernelGGL((fgp_sweep_kernel<KIND, C_NONE, true>), dim3(nblocks), dim3(NW * 64), 0, s, a);
    else hipLaunchKernelGGL((fgp_sweep_kernel<KIND, C_NONE, false>), dim3(nblocks), dim3(NW * 64), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fgp_sweep(const FgpPlainArgs& a, int kind, int constr, int batch, hipStream_t s) {
  if (a.T < 0 || a.T > kSweepMaxFuse || a.sweep_rows < 1 || kRW - 2 * a.halo < 1 || a.halo < a.T ||
      a.halo > a.T + 1 || (a.x != nullptr) != (a.halo == a.T + 1))
    return hipErrorInvalidValue;
  const int nblocks = a.tiles_x * a.tiles_y * batch;
  const bool mask = a.mask != nullptr;
  switch (kind) {
    case K1I: return launch_sweep_kind<K1I>(a, constr, mask, nblocks, s);
    case K1A: return launch_sweep_kind<K1A>(a, constr, mask, nblocks, s);
    case K2I: return launch_sweep_kind<K2I>(a, constr, mask, nblocks, s);
    default: return launch_sweep_kind<K2A>(a, constr, mask, nblocks, s);
  }
}

const void* fgp_sweep_batched_kernel_ptr(int constr) {
  return constr == C_MOD ? reinterpret_cast<const void*>(&fgp_sweep_batched_kernel<C_MOD>)
                         : reinterpret_cast<const void*>(&fgp_sweep_batched_kernel<C_NONE>);
}

}  // namespace ctv
