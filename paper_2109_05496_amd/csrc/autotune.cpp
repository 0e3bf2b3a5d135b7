// Autotuner of the fused forward kernel's launch configuration (tile shape and
// iterations fused per launch). For one problem, a plain call or a batched
// plan, it times every candidate configuration on the caller's data and stream
// and keeps the fastest in a process-wide table, which the automatic
// configuration of ctv_denoise, ctv_tiling, pr_prox_grad and
// ctv_batched_plan_create consults. Every configuration computes the same
// iterates bit for bit, so the table changes speed only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "ctv.h"
#include "ctv_host.hpp"
#include "ctv_kernels.hpp"

namespace ctv {
namespace {

struct TuneEntry {
  int T = 0, waves = 0, rows = 0;
  float ms = 0.0f;
  std::string what;  // readable description of the problem class
};

using TableKey = std::pair<std::string, uint64_t>;  // (device identity, problem key)

std::mutex g_mu;
std::map<TableKey, TuneEntry> g_table;
std::map<int, std::string> g_dev_ident;  // device ordinal -> identity (under g_mu)

// 64-bit FNV-1a over little-endian 8-byte words.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(long long v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((unsigned long long)v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  }
};

// Architecture name and CU count of the current device and the HIP runtime
// version ("" when there is no device).
// Caller holds g_mu.
std::string device_identity_locked() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return std::string();
  }
  auto it = g_dev_ident.find(dev);
  if (it != g_dev_ident.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return std::string();
  }
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess) {
    (void)hipGetLastError();
    rt = 0;
  }
  std::string id = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu/hip" +
                   std::to_string(rt);
  g_dev_ident[dev] = id;
  return id;
}

void record(uint64_t key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string id = device_identity_locked();
  if (!id.empty()) g_table[TableKey(id, key)] = e;
}

const char* kind_name(int k) {
  static const char* names[] = {"1i", "1a", "2i", "2a"};
  return (k >= 0 && k < 4) ? names[k] : "?";
}

struct Candidate {
  int waves, rows, T;
};

// Tile shapes worth trying and the largest fusion depth tried with each; the
// halo must leave at least one output row (T + 1 <= (rows - 1) / 2).
std::vector<Candidate> candidates(bool batched, int iters, bool single_tile) {
  struct Shape {
    int waves, rows, tmax;
  };
  // (kSweepShape, SH): the row-sweep tile with segments of SH output rows
  static const Shape plain_shapes[] = {{8, 8, 12}, {8, 4, 8}, {4, 8, 8}, {12, 4, 10}, {16, 4, 10},
                                       {kSweepShape, 144, kSweepMaxFuse}};
  static const Shape batched_shapes[] = {{8, 8, 12}, {8, 4, 8}, {12, 4, 10}, {16, 4, 10},
                                         {kSweepShape, 144, kSweepMaxFuse}};
  std::vector<Candidate> out;
  const int kcap = std::max(1, iters);
  auto add_shape = [&](const Shape& s) {
    const int rows = TileShape{s.waves, s.rows}.rows();
    const int hmax = (std::min(64, rows) - 1) / 2;
    const int tmax = std::min({s.tmax, hmax - 1, kMaxFuse, kcap});
    // an image inside one 8 x 8 tile runs in the single-tile kernel, which
    // ignores the fusion depth: one candidate stands for all of them
    if (single_tile && s.waves == 8 && s.rows == 8) {
      out.push_back(Candidate{8, 8, std::min(8, kcap)});
      return;
    }
    for (int T = std::min(2, tmax); T <= tmax; ++T) out.push_back(Candidate{s.waves, s.rows, T});
  };
  if (batched)
    for (const Shape& s : batched_shapes) add_shape(s);
  else
    for (const Shape& s : plain_shapes) add_shape(s);
  return out;
}

// Median of `reps` timed runs of fn() on stream s (after one untimed run).
template <class F>
ctv_status time_median(F fn, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms_out) {
  ctv_status st = fn();
  if (st) return st;
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    st = fn();
    if (st) return st;
    e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    t.push_back(ms);
  }
  std::sort(t.begin(), t.end());
  *ms_out = t[t.size() / 2];
  return CTV_OK;
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  hipError_t create() {
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    return e;
  }
};

ctv_status check_common(hipStream_t s, int reps) {
  if (reps < 1 || reps > 100) return fail(CTV_ERR_INVALID_ARG, "reps must lie in [1, 100]");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) return fail(CTV_ERR_INVALID_ARG, "autotuning cannot run under stream capture");
  return CTV_OK;
}

// Runs every candidate, fills the caller's result array and picks the fastest.
template <class Run>
ctv_status tune(const std::vector<Candidate>& cands, Run run, int reps, hipStream_t s, ctv_tuning* results,
                int max_results, int* num_results, ctv_tuning* best_out) {
  Events ev;
  hipError_t e = ev.create();
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  ctv_tuning best{0, 0, 0, 0.0f};
  int n = 0;
  for (const Candidate& c : cands) {
    float ms = 0.0f;
    ctv_status st = time_median([&] { return run(c); }, reps, s, ev.e0, ev.e1, &ms);
    if (st) return st;
    const ctv_tuning r{c.T, c.waves, c.rows, ms};
    if (results && n < max_results) results[n] = r;
    ++n;
    if (best.fuse == 0 || ms < best.ms) best = r;
  }
  if (num_results) *num_results = n;
  if (best_out) *best_out = best;
  return CTV_OK;
}

// --- text form of the table: one JSON object per line ----------------------

bool field_str(const std::string& line, const char* name, std::string* out) {
  const std::string pat = std::string("\"") + name + "\": \"";
  const size_t a = line.find(pat);
  if (a == std::string::npos) return false;
  const size_t b = line.find('"', a + pat.size());
  if (b == std::string::npos) return false;
  *out = line.substr(a + pat.size(), b - a - pat.size());
  return true;
}

bool field_num(const std::string& line, const char* name, double* out) {
  const std::string pat = std::string("\"") + name + "\": ";
  const size_t a = line.find(pat);
  if (a == std::string::npos) return false;
  const char* p = line.c_str() + a + pat.size();
  char* end = nullptr;
  const double v = std::strtod(p, &end);
  if (end == p) return false;
  *out = v;
  return true;
}

}  // namespace

uint64_t plain_tune_key(const ctv_params* p, int batch, int m, int n) {
  Fnv f;
  f.add(1);
  f.add(p->tv_kind);
  f.add(p->constraint);
  f.add(p->method);
  f.add(batch);
  f.add(m);
  f.add(n);
  f.add(p->iters);
  return f.h;
}

uint64_t batched_tune_key(const ctv_image_desc* d, int count, const ctv_params* common) {
  Fnv f;
  f.add(2);
  f.add(count);
  f.add(common->constraint);
  f.add(common->method);
  for (int i = 0; i < count; ++i) {
    f.add(d[i].m);
    f.add(d[i].n);
    f.add(d[i].lambda > 0.0f ? d[i].iters : 0);
    f.add(d[i].tv_kind);
    f.add(d[i].support_offset >= 0 ? 1 : 0);
  }
  return f.h;
}

bool tuned_lookup(uint64_t key, Tiling* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_table.empty()) return false;  // no device query while nothing was tuned
  const std::string id = device_identity_locked();
  if (id.empty()) return false;
  auto it = g_table.find(TableKey(id, key));
  if (it == g_table.end()) return false;
  out->T = it->second.T;
  out->shape.waves = it->second.waves;
  out->shape.rows_per_thread = it->second.rows;
  return true;
}

}  // namespace ctv

using namespace ctv;

extern "C" {

ctv_status ctv_autotune(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                        const float* lambda_host, const uint8_t* support, float* x, void* ws, size_t ws_bytes,
                        int32_t reps, ctv_tuning* results, int32_t max_results, int32_t* num_results,
                        ctv_tuning* best, ctv_stream_t stream) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (p->schedule == CTV_S_FLOW) return fail(CTV_ERR_INVALID_ARG, "autotuning covers the per-step schedule only");
  if (max_results < 0 || (max_results > 0 && !results)) return fail(CTV_ERR_INVALID_ARG, "results array missing");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = check_common(s, reps);
  if (st) return st;
  // the first candidate's call validates every other argument before any timing
  const std::vector<Candidate> cands = candidates(false, p->iters, m <= 64 && n <= 64);
  auto run = [&](const Candidate& c) {
    ctv_params q = *p;
    q.fuse = c.T;
    q.tile_waves = c.waves;
    q.tile_rows = c.rows;
    q.schedule = CTV_S_AUTO;
    return ctv_denoise(&q, batch, m, n, b, lambda_host, support, x, nullptr, nullptr, 0, nullptr, 0, nullptr, ws,
                       ws_bytes, stream);
  };
  ctv_tuning bst;
  st = tune(cands, run, reps, s, results, max_results, num_results, &bst);
  if (st) return st;
  if (best) *best = bst;
  TuneEntry e;
  e.T = bst.fuse;
  e.waves = bst.tile_waves;
  e.rows = bst.tile_rows;
  e.ms = bst.ms;
  e.what = std::string("plain ") + kind_name(p->tv_kind) + " constraint=" + std::to_string(p->constraint) +
           " method=" + std::to_string(p->method) + " batch=" + std::to_string(batch) + " m=" + std::to_string(m) +
           " n=" + std::to_string(n) + " K=" + std::to_string(p->iters);
  record(plain_tune_key(p, batch, m, n), e);
  return CTV_OK;
}

ctv_status ctv_batched_autotune(const ctv_image_desc* descs, int32_t count, const ctv_params* common,
                                const float* b_packed, const uint8_t* support_packed, float* x_packed, void* ws,
                                size_t ws_bytes, int32_t reps, ctv_tuning* results, int32_t max_results,
                                int32_t* num_results, ctv_tuning* best, ctv_stream_t stream) {
  ctv_status st = validate_params(common);
  if (st) return st;
  if (!descs || count < 1) return fail(CTV_ERR_INVALID_ARG, "need at least one image descriptor");
  if (max_results < 0 || (max_results > 0 && !results)) return fail(CTV_ERR_INVALID_ARG, "results array missing");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = check_common(s, reps);
  if (st) return st;
  int kmax = 0;
  for (int i = 0; i < count; ++i) kmax = std::max(kmax, descs[i].lambda > 0.0f ? descs[i].iters : 0);
  const std::vector<Candidate> cands = candidates(true, kmax, false);
  // each candidate's plan (tables, graph) is built once, outside the timed
  // launches, and destroyed after them
  Events ev;
  hipError_t he = ev.create();
  if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
  ctv_tuning bst{0, 0, 0, 0.0f};
  int nres = 0;
  for (const Candidate& c : cands) {
    ctv_params q = *common;
    q.fuse = c.T;
    q.tile_waves = c.waves;
    q.tile_rows = c.rows;
    ctv_batched_plan* plan = nullptr;
    st = ctv_batched_plan_create(descs, count, &q, &plan);
    if (st) return st;
    float ms = 0.0f;
    st = time_median([&] { return ctv_denoise_batched(plan, b_packed, support_packed, x_packed, ws, ws_bytes, stream); },
                     reps, s, ev.e0, ev.e1, &ms);
    he = hipStreamSynchronize(s);
    (void)ctv_batched_plan_destroy(plan);
    if (st) return st;
    if (he != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
    const ctv_tuning r{c.T, c.waves, c.rows, ms};
    if (results && nres < max_results) results[nres] = r;
    ++nres;
    if (bst.fuse == 0 || ms < bst.ms) bst = r;
  }
  if (num_results) *num_results = nres;
  if (best) *best = bst;
  TuneEntry e;
  e.T = bst.fuse;
  e.waves = bst.tile_waves;
  e.rows = bst.tile_rows;
  e.ms = bst.ms;
  e.what = "batched count=" + std::to_string(count) + " constraint=" + std::to_string(common->constraint) +
           " method=" + std::to_string(common->method) + " kmax=" + std::to_string(kmax);
  record(batched_tune_key(descs, count, common), e);
  return CTV_OK;
}

ctv_status ctv_tune_lookup(const ctv_params* p, int32_t batch, int32_t m, int32_t n, int32_t* found,
                           ctv_tuning* entry) {
  ctv_status st = validate_params(p);
  if (st) return st;
  if (!found) return fail(CTV_ERR_INVALID_ARG, "found is NULL");
  Tiling t;
  *found = tuned_lookup(plain_tune_key(p, batch, m, n), &t) ? 1 : 0;
  if (*found && entry) *entry = ctv_tuning{t.T, t.shape.waves, t.shape.rows_per_thread, 0.0f};
  return CTV_OK;
}

ctv_status ctv_batched_tune_lookup(const ctv_image_desc* descs, int32_t count, const ctv_params* common,
                                   int32_t* found, ctv_tuning* entry) {
  ctv_status st = validate_params(common);
  if (st) return st;
  if (!descs || count < 1) return fail(CTV_ERR_INVALID_ARG, "need at least one image descriptor");
  if (!found) return fail(CTV_ERR_INVALID_ARG, "found is NULL");
  Tiling t;
  *found = tuned_lookup(batched_tune_key(descs, count, common), &t) ? 1 : 0;
  if (*found && entry) *entry = ctv_tuning{t.T, t.shape.waves, t.shape.rows_per_thread, 0.0f};
  return CTV_OK;
}

ctv_status ctv_tune_cache_save(const char* path) {
  if (!path) return fail(CTV_ERR_INVALID_ARG, "path is NULL");
  std::ostringstream os;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_table) {
      char key[32];
      std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)kv.first.second);
      char ms[32];
      std::snprintf(ms, sizeof(ms), "%.6g", (double)kv.second.ms);
      os << "{\"arch\": \"" << kv.first.first << "\", \"key\": \"" << key << "\", \"fuse\": " << kv.second.T
         << ", \"tile_waves\": " << kv.second.waves << ", \"tile_rows\": " << kv.second.rows << ", \"ms\": " << ms
         << ", \"what\": \"" << kv.second.what << "\"}\n";
    }
  }
  std::ofstream f(path, std::ios::out | std::ios::trunc);
  if (!f) return fail(CTV_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
  f << os.str();
  f.close();
  if (!f) return fail(CTV_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
  return CTV_OK;
}

ctv_status ctv_tune_cache_load(const char* path) {
  if (!path) return fail(CTV_ERR_INVALID_ARG, "path is NULL");
  std::ifstream f(path);
  if (!f) return fail(CTV_ERR_INVALID_ARG, std::string("cannot open ") + path);
  std::vector<std::pair<TableKey, TuneEntry>> parsed;
  std::string line;
  int lineno = 0;
  while (std::getline(f, line)) {
    ++lineno;
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    std::string arch, key, what;
    double T = 0, w = 0, r = 0, ms = 0;
    const bool ok = field_str(line, "arch", &arch) && field_str(line, "key", &key) && field_num(line, "fuse", &T) &&
                    field_num(line, "tile_waves", &w) && field_num(line, "tile_rows", &r) &&
                    field_num(line, "ms", &ms);
    char* end = nullptr;
    const unsigned long long k = ok ? std::strtoull(key.c_str(), &end, 16) : 0;
    // range and integrality are checked on the doubles, before any conversion
    auto small_int = [](double v, int lo, int hi) { return v >= lo && v <= hi && v == std::floor(v); };
    const bool nums = small_int(T, 1, kMaxFuse) && (small_int(w, 1, 64) || w == kSweepShape) && small_int(r, 1, 256);
    const TileShape ts{nums ? (int)w : 0, nums ? (int)r : 0};
    if (!ok || key.empty() || (end && *end) || arch.empty() || !nums || !valid_tile_shape(ts))
      return fail(CTV_ERR_INVALID_ARG, std::string(path) + ":" + std::to_string(lineno) + ": malformed tuning entry");
    (void)field_str(line, "what", &what);
    TuneEntry e;
    e.T = (int)T;
    e.waves = ts.waves;
    e.rows = ts.rows_per_thread;
    e.ms = (float)ms;
    e.what = what;
    parsed.emplace_back(TableKey(arch, (uint64_t)k), e);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : parsed) g_table[kv.first] = kv.second;
  return CTV_OK;
}

ctv_status ctv_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  return CTV_OK;
}

int32_t ctv_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int32_t)g_table.size();
}

}  // extern "C"
