// Batched ragged denoising: a plan holds the device descriptor table, the
// float64-derived momentum table, one tile list per fused step and a HIP graph
// with one kernel node per step (one workgroup per tile of the step, so the
// hardware dispatcher balances the load). Executing the plan is one
// hipGraphLaunch; pointers that change between calls are patched into the
// instantiated graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>
#include <string>
#include <vector>

#include "ctv.h"
#include "ctv_host.hpp"
#include "ctv_kernels.hpp"

using namespace ctv;

struct ctv_batched_plan {
  int count = 0;
  int constraint = 0;
  Tiling tiling{};
  int kmax = 0;
  long long total_px = 0;
  bool any_support = false;
  BatchImage* d_images = nullptr;
  BatchTile* d_tiles = nullptr;
  float* d_beta = nullptr;
  std::vector<int> step_offset, step_count;
  std::vector<FgpBatchedArgs> args;
  std::vector<hipGraphNode_t> nodes;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* func = nullptr;
  int block = 0;
  // live-tile skipping for images with a support (see ctv_denoise): scan and
  // compaction nodes ahead of the steps
  int nflags = 0;
  BatchGeom* d_geoms = nullptr;
  int* d_geo_of = nullptr;
  int* d_flags = nullptr;
  int* d_lists = nullptr;
  int* d_counts = nullptr;
  int* d_step_offset = nullptr;
  int* d_step_count = nullptr;
  BatchScanArgs scan_args{};
  BatchCompactArgs compact_args{};
  hipGraphNode_t scan_node = nullptr, compact_node = nullptr;
  const float* b = nullptr;
  const uint8_t* support = nullptr;
  float* x = nullptr;
  void* ws = nullptr;
};

namespace {

void release(ctv_batched_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_images) (void)hipFree(p->d_images);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  if (p->d_beta) (void)hipFree(p->d_beta);
  for (void* q : {(void*)p->d_geoms, (void*)p->d_geo_of, (void*)p->d_flags, (void*)p->d_lists, (void*)p->d_counts,
                  (void*)p->d_step_offset, (void*)p->d_step_count})
    if (q) (void)hipFree(q);
  delete p;
}

size_t batched_ws_bytes(const ctv_batched_plan* p) { return 2 * (size_t)p->total_px * 32; }

void fill_args(ctv_batched_plan* p) {
  float* buf0 = static_cast<float*>(p->ws);
  float* buf1 = buf0 ? buf0 + (size_t)p->total_px * 8 : nullptr;
  for (size_t s = 0; s < p->args.size(); ++s) {
    FgpBatchedArgs& a = p->args[s];
    a.tiles = p->d_tiles + p->step_offset[s];
    a.ntiles = p->step_count[s];
    a.images = p->d_images;
    a.beta_table = p->d_beta;
    a.b = p->b;
    a.support = p->support;
    a.st_out = (s % 2 == 0) ? buf0 : buf1;
    a.st_in = (s == 0) ? nullptr : ((s % 2 == 1) ? buf0 : buf1);
    a.x = p->x;
    a.k0 = (int)s * p->tiling.T;
    a.T = p->tiling.T;
    a.live = p->nflags ? p->d_lists + p->step_offset[s] : nullptr;
    a.live_count = p->nflags ? p->d_counts + s : nullptr;
    a.sweep_rows = p->tiling.shape.sweep() ? p->tiling.shape.rows_per_thread : 0;
  }
  BatchScanArgs& sa = p->scan_args;
  sa.images = p->d_images;
  sa.geoms = p->d_geoms;
  sa.geo_of = p->d_geo_of;
  sa.support = p->support;
  sa.st0 = buf0;
  sa.st1 = buf1;
  sa.x = p->x;
  sa.flags = p->d_flags;
  sa.rows = p->tiling.shape.rows();
  sa.sweep_oh = p->tiling.shape.sweep() ? p->tiling.shape.rows_per_thread : 0;
  BatchCompactArgs& ca = p->compact_args;
  ca.tiles = p->d_tiles;
  ca.step_offset = p->d_step_offset;
  ca.step_count = p->d_step_count;
  ca.flags = p->d_flags;
  ca.lists = p->d_lists;
  ca.counts = p->d_counts;
}

hipKernelNodeParams aux_params(const void* func, int grid, int block, void** kp) {
  hipKernelNodeParams np;
  std::memset(&np, 0, sizeof(np));
  np.func = const_cast<void*>(func);
  np.gridDim = dim3((unsigned)grid);
  np.blockDim = dim3((unsigned)block);
  np.kernelParams = kp;
  return np;
}

hipKernelNodeParams node_params(ctv_batched_plan* p, size_t s, void** kp) {
  hipKernelNodeParams np;
  std::memset(&np, 0, sizeof(np));
  np.func = const_cast<void*>(p->func);
  np.gridDim = dim3((unsigned)std::max(1, p->step_count[s]));
  np.blockDim = dim3((unsigned)p->block);
  np.sharedMemBytes = 0;
  np.kernelParams = kp;
  np.extra = nullptr;
  return np;
}

ctv_status build_graph(ctv_batched_plan* p) {
  hipError_t e = hipGraphCreate(&p->graph, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
  p->nodes.assign(p->args.size(), nullptr);
  if (p->nflags) {
    void* kp0[] = {&p->scan_args};
    hipKernelNodeParams n0 = aux_params(batched_scan_kernel_ptr(), p->nflags, 256, kp0);
    e = hipGraphAddKernelNode(&p->scan_node, p->graph, nullptr, 0, &n0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode (live scan)");
    void* kp1[] = {&p->compact_args};
    hipKernelNodeParams n1 = aux_params(batched_compact_kernel_ptr(), (int)p->args.size(), 1024, kp1);
    e = hipGraphAddKernelNode(&p->compact_node, p->graph, &p->scan_node, 1, &n1);
    if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode (live lists)");
  }
  for (size_t s = 0; s < p->args.size(); ++s) {
    void* kp[] = {&p->args[s]};
    hipKernelNodeParams np = node_params(p, s, kp);
    const hipGraphNode_t* dep = s ? &p->nodes[s - 1] : (p->nflags ? &p->compact_node : nullptr);
    e = hipGraphAddKernelNode(&p->nodes[s], p->graph, dep, dep ? 1 : 0, &np);
    if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode");
  }
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return CTV_OK;
}

}  // namespace

extern "C" {

ctv_status ctv_batched_plan_create(const ctv_image_desc* descs, int32_t count, const ctv_params* common,
                                   ctv_batched_plan** plan_out) {
  if (!plan_out) return fail(CTV_ERR_INVALID_ARG, "plan output pointer is NULL");
  *plan_out = nullptr;
  if (!descs || count < 1) return fail(CTV_ERR_INVALID_ARG, "need at least one image descriptor");
  ctv_status st = validate_params(common);
  if (st) return st;
  std::vector<BatchImage> imgs((size_t)count);
  std::vector<std::pair<long long, long long>> spans;
  int kmax = 0;
  long long total = 0;
  bool any_support = false;
  for (int i = 0; i < count; ++i) {
    const ctv_image_desc& d = descs[i];
    if (d.m < 1 || d.n < 1) return fail(CTV_ERR_INVALID_ARG, "image " + std::to_string(i) + ": m and n must be >= 1");
    if (d.offset < 0) return fail(CTV_ERR_INVALID_ARG, "image " + std::to_string(i) + ": negative offset");
    if (d.tv_kind < CTV_TV_1I || d.tv_kind > CTV_TV_2A) return fail(CTV_ERR_INVALID_ARG, "image " + std::to_string(i) + ": unknown tv_kind");
    if (!(d.alpha >= 0.0f && d.alpha <= 1.0f)) return fail(CTV_ERR_INVALID_ARG, "image " + std::to_string(i) + ": alpha outside [0, 1]");
    if (d.iters < 0 || d.iters > (1 << 24)) return fail(CTV_ERR_INVALID_ARG, "image " + std::to_string(i) + ": iters out of range");
    if (d.support_offset < -1) return fail(CTV_ERR_INVALID_ARG, "image " + std::to_string(i) + ": bad support_offset");
    st = validate_lambda(d.lambda);
    if (st) return st;
    const long long px = (long long)d.m * d.n;
    BatchImage& b = imgs[(size_t)i];
    b.offset = d.offset;
    b.support_offset = d.support_offset;
    b.m = d.m;
    b.n = d.n;
    b.kind = d.tv_kind;
    b.iters = d.lambda > 0.0f ? d.iters : 0;
    b.lam = d.lambda;
    b.c = step_of(d.lambda);
    b.R = make_radii(d.tv_kind, d.alpha);
    kmax = std::max(kmax, b.iters);
    total = std::max(total, d.offset + px);
    any_support = any_support || d.support_offset >= 0;
    spans.emplace_back(d.offset, d.offset + px);
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second) return fail(CTV_ERR_INVALID_ARG, "images overlap in the packed buffer");

  Tiling tl;
  ctv_params tp = *common;
  tp.iters = std::max(kmax, 1);
  st = choose_tiling(&tp, 1, 1, count, &tl);
  if (st) return st;
  if (common->fuse == 0 && common->tile_waves == 0 && common->tile_rows == 0) {
    Tiling tuned;
    if (tuned_lookup(batched_tune_key(descs, count, common), &tuned) &&
        fgp_batched_kernel_ptr(common->constraint, tuned.shape)) {
      clamp_fuse(&tuned, tp.iters);
      tl = tuned;
    }
  }
  ctv_batched_plan* p = new ctv_batched_plan();
  p->count = count;
  p->constraint = common->constraint;
  p->tiling = tl;
  p->kmax = kmax;
  p->total_px = total;
  p->any_support = any_support;
  p->func = fgp_batched_kernel_ptr(common->constraint, tl.shape);
  if (!p->func) {
    release(p);
    return fail(CTV_ERR_UNSUPPORTED, "the batched kernel supports the 8x8, 8x4 and 16x4 column tiles and the row sweep");
  }
  p->block = tl.shape.threads();
  const int T = tl.T;

  // per-step tile lists; tiles of images with a support (and iterations) get a
  // live flag of their (image, tiling) pair
  const int steps = std::max(1, (kmax + T - 1) / T);
  std::vector<BatchTile> tiles;
  std::vector<BatchGeom> geoms;
  std::vector<int> geo_of;
  std::map<std::tuple<int, int, int>, int> geo_index;
  std::vector<char> image_zeroed((size_t)count, 0);
  for (int s = 0; s < steps; ++s) {
    const int k0 = s * T;
    p->step_offset.push_back((int)tiles.size());
    for (int i = 0; i < count; ++i) {
      const BatchImage& b = imgs[(size_t)i];
      if (!(b.iters > k0 || (b.iters == 0 && k0 == 0))) continue;
      const int Ti = std::min(T, b.iters - k0);
      const bool last = (k0 + Ti == b.iters);
      const int H = std::max(1, Ti + (last ? 1 : 0));
      const int ow = 64 - 2 * H, oh = tl.shape.out_rows(H);
      const int tx = (b.n + ow - 1) / ow, ty = (b.m + oh - 1) / oh;
      int base = -1;
      if (b.support_offset >= 0 && b.iters > 0) {
        const auto key = std::make_tuple(i, H, last ? 1 : 0);
        auto it = geo_index.find(key);
        if (it == geo_index.end()) {
          BatchGeom g{};
          g.image = i;
          g.halo = H;
          g.tiles_x = tx;
          g.tiles_y = ty;
          g.flag_base = (int)geo_of.size();
          g.zero_st = image_zeroed[(size_t)i] ? 0 : 1;
          g.zero_x = last ? 1 : 0;
          image_zeroed[(size_t)i] = 1;
          geo_of.insert(geo_of.end(), (size_t)tx * ty, (int)geoms.size());
          it = geo_index.emplace(key, (int)geoms.size()).first;
          geoms.push_back(g);
        }
        base = geoms[(size_t)it->second].flag_base;
      }
      for (int y = 0; y < ty; ++y)
        for (int x = 0; x < tx; ++x) tiles.push_back(BatchTile{i, x, y, base < 0 ? -1 : base + y * tx + x});
    }
    p->step_count.push_back((int)tiles.size() - p->step_offset.back());
  }
  if (tiles.size() > (size_t)0x7fffffff) {
    release(p);
    return fail(CTV_ERR_INVALID_ARG, "batch too large");
  }
  std::vector<float> beta;
  momentum_table(common->method, steps * T + kMaxFuse + 1, beta);

  hipError_t e = hipMalloc(&p->d_images, imgs.size() * sizeof(BatchImage));
  if (e == hipSuccess) e = hipMalloc(&p->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(BatchTile));
  if (e == hipSuccess) e = hipMalloc(&p->d_beta, beta.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(p->d_images, imgs.data(), imgs.size() * sizeof(BatchImage), hipMemcpyHostToDevice);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_beta, beta.data(), beta.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess && !geoms.empty()) {
    p->nflags = (int)geo_of.size();
    const size_t nt = std::max<size_t>(1, tiles.size());
    e = hipMalloc(&p->d_geoms, geoms.size() * sizeof(BatchGeom));
    if (e == hipSuccess) e = hipMalloc(&p->d_geo_of, geo_of.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_flags, geo_of.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_lists, nt * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_counts, (size_t)steps * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_step_offset, (size_t)steps * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_step_count, (size_t)steps * sizeof(int));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_geoms, geoms.data(), geoms.size() * sizeof(BatchGeom), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_geo_of, geo_of.data(), geo_of.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_step_offset, p->step_offset.data(), (size_t)steps * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_step_count, p->step_count.data(), (size_t)steps * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    release(p);
    return hip_fail(e, "batched plan setup");
  }
  p->args.resize((size_t)steps);
  *plan_out = p;
  return CTV_OK;
}

ctv_status ctv_batched_workspace_size(const ctv_batched_plan* p, size_t* ws_bytes) {
  if (!p || !ws_bytes) return fail(CTV_ERR_INVALID_ARG, "plan and ws_bytes must be non-NULL");
  *ws_bytes = batched_ws_bytes(p);
  return CTV_OK;
}

ctv_status ctv_denoise_batched(ctv_batched_plan* p, const float* b, const uint8_t* support, float* x, void* ws,
                               size_t ws_bytes, ctv_stream_t stream) {
  if (!p) return fail(CTV_ERR_INVALID_ARG, "plan is NULL");
  if (!b || !x) return fail(CTV_ERR_INVALID_ARG, "b and x must be non-NULL");
  if (b == x) return fail(CTV_ERR_INVALID_ARG, "x must not alias b");
  if (p->any_support && !support) return fail(CTV_ERR_INVALID_ARG, "an image has a support mask but support is NULL");
  if (!ws) return fail(CTV_ERR_INVALID_ARG, "ws is NULL");
  if (ws_bytes < batched_ws_bytes(p)) return fail(CTV_ERR_WORKSPACE, "workspace too small: need " + std::to_string(batched_ws_bytes(p)) + " bytes");
  const bool changed = b != p->b || support != p->support || x != p->x || ws != p->ws;
  p->b = b;
  p->support = support;
  p->x = x;
  p->ws = ws;
  if (!p->exec) {
    fill_args(p);
    ctv_status st = build_graph(p);
    if (st) return st;
  } else if (changed) {
    fill_args(p);
    if (p->nflags) {
      void* kp0[] = {&p->scan_args};
      hipKernelNodeParams n0 = aux_params(batched_scan_kernel_ptr(), p->nflags, 256, kp0);
      hipError_t e = hipGraphExecKernelNodeSetParams(p->exec, p->scan_node, &n0);
      if (e != hipSuccess) return hip_fail(e, "hipGraphExecKernelNodeSetParams (live scan)");
    }
    for (size_t s = 0; s < p->args.size(); ++s) {
      void* kp[] = {&p->args[s]};
      hipKernelNodeParams np = node_params(p, s, kp);
      hipError_t e = hipGraphExecKernelNodeSetParams(p->exec, p->nodes[s], &np);
      if (e != hipSuccess) return hip_fail(e, "hipGraphExecKernelNodeSetParams");
    }
  }
  hipError_t e = hipGraphLaunch(p->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return CTV_OK;
}

ctv_status ctv_batched_plan_tiling(const ctv_batched_plan* p, int32_t* fuse_out, int32_t* tile_waves_out,
                                   int32_t* tile_rows_out) {
  if (!p) return fail(CTV_ERR_INVALID_ARG, "plan is NULL");
  if (fuse_out) *fuse_out = p->tiling.T;
  if (tile_waves_out) *tile_waves_out = p->tiling.shape.waves;
  if (tile_rows_out) *tile_rows_out = p->tiling.shape.rows_per_thread;
  return CTV_OK;
}

ctv_status ctv_batched_plan_destroy(ctv_batched_plan* p) {
  if (!p) return fail(CTV_ERR_INVALID_ARG, "plan is NULL");
  release(p);
  return CTV_OK;
}

}  // extern "C"
