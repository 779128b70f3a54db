// Host side of the ragged batch: validation, per-class steering tables,
// longest-first ordering, route choice, hipGraph capture of the persistent
// launch, and the autotuner that times tile and route candidates on the
// batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "ragged.h"

namespace ba {
namespace {

struct Ragged {
  const Plan* plan = nullptr;
  int device = 0;
  std::vector<ba_trial> desc;          // caller's order
  std::vector<int> cls, tuned_route;   // per trial
  int kmax = 1;
  const float2* Y = nullptr;
  int64_t pool_need = 0;               // complex elements the pool must hold
  float* P = nullptr;
  int32_t* idx = nullptr;
  float* val = nullptr;
  double* refined = nullptr;
  float4* X[kRaggedClasses] = {};
  int nchunk[kRaggedClasses] = {};
  int wr[kRaggedClasses] = {1, 1, 2, 4, 8};
  bool pack[kRaggedPackClasses] = {true, true, true};  // small classes one trial per wave (tuned)
  int n_wg_items = 0;                            // of the uploaded full batch
  std::map<std::pair<int, int>, int> route_table;  // (class, log2 T bucket) -> route
  RItem* d_items = nullptr;
  RArgs* d_args = nullptr;        // arguments of the captured launch (device copy)
  RArgs* d_args_probe = nullptr;  // arguments of autotuner probes
  int32_t* d_counter = nullptr;
  int n_wg = 1;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int class_of(int M) { return M <= 8 ? 0 : M <= 16 ? 1 : M <= 32 ? 2 : M <= 64 ? 3 : 4; }
int bucket_of(int T) {
  int b = 0;
  while ((2 << b) <= T) ++b;
  return b;
}

// The snapshot route needs 2 * ceil8(T) <= 2 * Mp rows.
bool snapshot_allowed(int T, int cls) { return ((T + 7) & ~7) <= (8 << cls); }

int route_for(const Ragged& r, size_t i) {
  const ba_trial& d = r.desc[i];
  const int c = r.cls[i];
  if (d.route == BA_ROUTE_COV) return kRouteCov;
  if (d.route == BA_ROUTE_SNAPSHOTS) return kRouteSnap;
  auto it = r.route_table.find({c, bucket_of(d.n_snap)});
  if (it != r.route_table.end()) return (it->second == kRouteSnap && snapshot_allowed(d.n_snap, c)) ? kRouteSnap : kRouteCov;
  return (d.n_snap < d.n_elem && snapshot_allowed(d.n_snap, c)) ? kRouteSnap : kRouteCov;
}

// work estimate for the longest-first order (MFMA flops of the padded class
// plus the covariance on the vector units, weighted by their relative rates)
double cost_of(const Ragged& r, size_t i, int route) {
  const ba_trial& d = r.desc[i];
  const double Mp = double(8 << r.cls[i]), G = double(r.plan->G);
  if (route == kRouteSnap) return 8.0 * Mp * ((d.n_snap + 7) & ~7) * G;
  return 8.0 * Mp * Mp * G + 2.0 * 4.0 * double(d.n_elem) * d.n_elem * d.n_snap;
}

// Items in processing order: whole-workgroup items longest first, then the
// packed ones (longest first among themselves, eight per ticket).
struct ItemList {
  std::vector<RItem> items;
  int n_wg = 0;
};

// A trial runs packed when its class is packed, it takes the covariance route
// and the grid is 1-D (the packed path keeps no spectrum row).
bool packed(const Ragged& r, const RItem& it, bool force_wg) {
  return !force_wg && it.cls < kRaggedPackClasses && r.pack[it.cls] && it.route == kRouteCov &&
         r.plan->shape1 == 1;
}

ItemList make_items(const Ragged& r, const std::vector<size_t>& which, const int* force_route,
                    bool force_wg = false) {
  std::vector<RItem> items;
  items.reserve(which.size());
  std::vector<double> cost;
  for (size_t i : which) {
    const ba_trial& d = r.desc[i];
    RItem it;
    it.y_off = d.y_offset;
    it.trial = int32_t(i);
    it.M = d.n_elem;
    it.T = d.n_snap;
    it.K = d.k;
    it.cls = r.cls[i];
    it.route = force_route ? *force_route : route_for(r, i);
    if (it.route == kRouteSnap && !snapshot_allowed(it.T, it.cls)) it.route = kRouteCov;
    items.push_back(it);
    cost.push_back(cost_of(r, i, it.route));
  }
  std::vector<size_t> ord(items.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  // whole-workgroup items first; the order within each group is kept
  std::stable_partition(ord.begin(), ord.end(), [&](size_t a) { return !packed(r, items[a], force_wg); });
  ItemList out;
  out.items.resize(items.size());
  for (size_t i = 0; i < ord.size(); ++i) {
    out.items[i] = items[ord[i]];
    if (!packed(r, out.items[i], force_wg)) out.n_wg = int(i) + 1;
  }
  return out;
}

RArgs make_args(const Ragged& r, const RItem* d_items, int n, int n_wg_items) {
  RArgs a{};
  a.items = d_items;
  a.n_items = n;
  a.n_wg_items = n_wg_items;
  a.n_units = n_wg_items + (n - n_wg_items + kRaggedPackWaves - 1) / kRaggedPackWaves;
  a.Y = r.Y;
  for (int c = 0; c < kRaggedClasses; ++c) {
    a.X[c] = r.X[c];
    a.nchunk[c] = r.nchunk[c];
    a.wr[c] = r.wr[c];
  }
  a.G = r.plan->G;
  a.s1 = r.plan->shape1;
  a.rows = r.plan->rows;
  a.wrap0 = r.plan->wrap0;
  a.ndim = r.plan->ndim;
  a.kmax = r.kmax;
  a.P = r.P;
  a.idx = r.idx;
  a.val = r.val;
  a.refined = r.refined;
  a.counter = r.d_counter;
  return a;
}

hipError_t upload_items(Ragged& r, const ItemList& list) {
  r.n_wg_items = list.n_wg;
  return hipMemcpy(r.d_items, list.items.data(), list.items.size() * sizeof(RItem), hipMemcpyHostToDevice);
}

hipError_t capture(Ragged& r) {
  if (r.exec) {
    (void)hipGraphExecDestroy(r.exec);
    r.exec = nullptr;
  }
  if (r.graph) {
    (void)hipGraphDestroy(r.graph);
    r.graph = nullptr;
  }
  const RArgs a = make_args(r, r.d_items, int(r.desc.size()), r.n_wg_items);
  hipError_t e = hipMemcpy(r.d_args, &a, sizeof(RArgs), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(r.cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  // the ticket counter is cleared by a kernel, not a memset node
  hipError_t e1 = launch_ragged_reset(r.d_counter, r.cap);
  hipError_t e2 = e1 == hipSuccess ? launch_ragged(r.d_args, r.n_wg, r.cap) : e1;
  e = hipStreamEndCapture(r.cap, &r.graph);
  if (e2 != hipSuccess) return e2;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&r.exec, r.graph, nullptr, nullptr, 0);
}

// one direct (uncaptured) launch over a subset, timed with events
hipError_t time_subset(Ragged& r, const ItemList& list, int repeats, float* ms) {
  const std::vector<RItem>& items = list.items;
  RItem* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(1, items.size()) * sizeof(RItem));
  if (e != hipSuccess) return e;
  e = hipMemcpy(d, items.data(), items.size() * sizeof(RItem), hipMemcpyHostToDevice);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const RArgs a = make_args(r, d, int(items.size()), list.n_wg);
  if (e == hipSuccess) e = hipMemcpy(r.d_args_probe, &a, sizeof(RArgs), hipMemcpyHostToDevice);
  const int nwg = std::max(1, std::min<int>(r.n_wg, a.n_units));
  float best = 1e30f;
  for (int rep = 0; e == hipSuccess && rep < repeats + 1; ++rep) {
    e = launch_ragged_reset(r.d_counter, r.cap);
    if (e == hipSuccess) e = hipEventRecord(e0, r.cap);
    if (e == hipSuccess) e = launch_ragged(r.d_args_probe, nwg, r.cap);
    if (e == hipSuccess) e = hipEventRecord(e1, r.cap);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (rep > 0) best = std::min(best, t);  // the first launch is a warm-up
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  *ms = best;
  return e;
}

std::string device_key(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string n = prop.gcnArchName;
  for (char& c : n)
    if (c == ' ' || c == '|') c = '_';
  return n + ":" + std::to_string(prop.multiProcessorCount);
}

}  // namespace
}  // namespace ba

using namespace ba;

struct ba_ragged_s : public ba::Ragged {};

static ba_status rg_arg(const char* fn, const std::string& what) {
  set_error(std::string(fn) + ": " + what);
  return BA_ERR_ARG;
}

static ba_status rg_dev(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return e == hipErrorOutOfMemory ? BA_ERR_NOMEM : BA_ERR_DEVICE;
}

static void rg_free(ba_ragged r) {
  if (!r) return;
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  if (r->graph) (void)hipGraphDestroy(r->graph);
  if (r->cap) (void)hipStreamDestroy(r->cap);
  for (int c = 0; c < kRaggedClasses; ++c)
    if (r->X[c]) (void)hipFree(r->X[c]);
  if (r->d_items) (void)hipFree(r->d_items);
  if (r->d_args) (void)hipFree(r->d_args);
  if (r->d_args_probe) (void)hipFree(r->d_args_probe);
  if (r->d_counter) (void)hipFree(r->d_counter);
  delete r;
}

extern "C" {

ba_status ba_ragged_create(ba_ragged* out, ba_plan plan, int32_t n_trials, const ba_trial* desc,
                           int32_t kmax, const void* Y_pool, int64_t pool_elems, float* P,
                           int32_t* idx, float* val, double* refined) {
  static const char* fn = "ba_ragged_create";
  if (!out) return rg_arg(fn, "out is NULL");
  *out = nullptr;
  if (!plan) return rg_arg(fn, "plan is NULL");
  const Plan& q = *static_cast<const Plan*>(plan);
  if (n_trials < 1) return rg_arg(fn, "n_trials >= 1 required");
  if (!desc) return rg_arg(fn, "desc is NULL");
  if (kmax < 1 || kmax > kRaggedMaxPeaks) return rg_arg(fn, "kmax must be in [1, 8]");
  if (q.G > kRaggedMaxGrid) return rg_arg(fn, "the ragged path needs a grid of at most 16384 points");
  if (q.precision != BA_PREC_F32) return rg_arg(fn, "the ragged path runs in FP32 (BA_PREC_F32 plan)");
  if (!Y_pool || pool_elems < 1) return rg_arg(fn, "Y_pool is NULL or empty");
  if (!idx || !val) return rg_arg(fn, "idx and val are required");
  const int mmax = std::min(q.M, 128);
  for (int32_t i = 0; i < n_trials; ++i) {
    const ba_trial& d = desc[i];
    std::ostringstream w;
    w << "trial " << i << ": ";
    if (d.n_elem < 1 || d.n_elem > mmax) return rg_arg(fn, w.str() + "n_elem must be in [1, min(128, plan elements)]");
    if (d.n_snap < 1) return rg_arg(fn, w.str() + "n_snap must be >= 1");
    if (d.k < 1 || d.k > kmax) return rg_arg(fn, w.str() + "k must be in [1, kmax]");
    if (d.route < BA_ROUTE_AUTO || d.route > BA_ROUTE_SNAPSHOTS) return rg_arg(fn, w.str() + "unknown route");
    if (d.route == BA_ROUTE_SNAPSHOTS && !snapshot_allowed(d.n_snap, class_of(d.n_elem)))
      return rg_arg(fn, w.str() + "the snapshot route needs n_snap <= the padded element count");
    if (d.y_offset < 0 || d.y_offset + int64_t(d.n_elem) * d.n_snap > pool_elems)
      return rg_arg(fn, w.str() + "snapshot block outside the pool");
  }

  ba_ragged r = new (std::nothrow) ba_ragged_s();
  if (!r) return rg_arg(fn, "host allocation failed");
  r->plan = &q;
  r->device = q.device;
  r->desc.assign(desc, desc + n_trials);
  r->kmax = kmax;
  r->Y = static_cast<const float2*>(Y_pool);
  for (int32_t i = 0; i < n_trials; ++i)
    r->pool_need = std::max(r->pool_need, desc[i].y_offset + int64_t(desc[i].n_elem) * desc[i].n_snap);
  r->P = P;
  r->idx = idx;
  r->val = val;
  r->refined = refined;
  r->cls.resize(n_trials);
  bool present[kRaggedClasses] = {};
  for (int32_t i = 0; i < n_trials; ++i) present[r->cls[i] = class_of(desc[i].n_elem)] = true;

  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(r->device);
  hipError_t e = ragged_prepare();
  for (int c = 0; e == hipSuccess && c < kRaggedClasses; ++c) {
    if (!present[c]) continue;
    const int Mp = 8 << c;
    const int NB = ragged_blocks_per_chunk(c);
    const int64_t Gb = (q.G + 15) / 16;
    r->nchunk[c] = int((Gb + NB - 1) / NB);
    std::vector<float> x = plan_x_table(q, std::min(Mp, q.M), Mp, int64_t(r->nchunk[c]) * NB);
    e = hipMalloc(&r->X[c], x.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(r->X[c], x.data(), x.size() * sizeof(float), hipMemcpyHostToDevice);
  }
  int ncu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, r->device);
  r->n_wg = std::max(1, std::min(ncu, n_trials));
  if (e == hipSuccess) e = hipMalloc(&r->d_items, size_t(n_trials) * sizeof(RItem));
  if (e == hipSuccess) e = hipMalloc(&r->d_counter, 256);
  if (e == hipSuccess) e = hipMalloc(&r->d_args, sizeof(RArgs));
  if (e == hipSuccess) e = hipMalloc(&r->d_args_probe, sizeof(RArgs));
  if (e == hipSuccess) e = hipStreamCreate(&r->cap);
  if (e == hipSuccess) {
    std::vector<size_t> all(n_trials);
    for (int32_t i = 0; i < n_trials; ++i) all[i] = size_t(i);
    e = upload_items(*r, make_items(*r, all, nullptr));
  }
  if (e == hipSuccess) e = capture(*r);
  (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    ba_status st = rg_dev(fn, e);
    rg_free(r);
    return st;
  }
  *out = r;
  return BA_OK;
}

ba_status ba_ragged_bind(ba_ragged r, const void* Y_pool, int64_t pool_elems, float* P, int32_t* idx, float* val,
                         double* refined, void* stream) {
  static const char* fn = "ba_ragged_bind";
  if (!r) return rg_arg(fn, "handle is NULL");
  if (!Y_pool || pool_elems < r->pool_need) return rg_arg(fn, "Y_pool is NULL or smaller than the trials' blocks");
  if (!idx || !val) return rg_arg(fn, "idx and val are required");
  r->Y = static_cast<const float2*>(Y_pool);
  r->P = P;
  r->idx = idx;
  r->val = val;
  r->refined = refined;
  // the captured launch reads its arguments from device memory: rewriting
  // the buffer fields there (in stream order) retargets every later replay
  const hipError_t e = launch_ragged_bind(r->d_args, r->Y, P, idx, val, refined, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : rg_dev(fn, e);
}

ba_status ba_ragged_launch(ba_ragged r, void* stream) {
  if (!r) return rg_arg("ba_ragged_launch", "handle is NULL");
  hipError_t e = hipGraphLaunch(r->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : rg_dev("ba_ragged_launch", e);
}

ba_status ba_ragged_routes(ba_ragged r, int32_t* routes) {
  if (!r || !routes) return rg_arg("ba_ragged_routes", "null argument");
  for (size_t i = 0; i < r->desc.size(); ++i) {
    int rt = route_for(*r, i);
    if (rt == kRouteSnap && !snapshot_allowed(r->desc[i].n_snap, r->cls[i])) rt = kRouteCov;
    routes[i] = rt;
  }
  return BA_OK;
}

ba_status ba_ragged_autotune(ba_ragged r, const char* cache_path, int32_t repeats, int32_t max_probe) {
  static const char* fn = "ba_ragged_autotune";
  if (!r) return rg_arg(fn, "handle is NULL");
  if (repeats < 1 || max_probe < 1) return rg_arg(fn, "repeats and max_probe must be >= 1");
  const std::string dev = device_key(r->device) + "|G" + std::to_string(r->plan->G);
  std::map<std::string, int> cache;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string key;
    int v;
    while (in >> key >> v) cache[key] = v;
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(r->device);
  hipError_t e = hipSuccess;
  const size_t n = r->desc.size();
  // 1. tiles: waves along rows, per size class
  for (int c = 0; e == hipSuccess && c < kRaggedClasses; ++c) {
    std::vector<size_t> which;
    for (size_t i = 0; i < n && int(which.size()) < max_probe; ++i)
      if (r->cls[i] == c) which.push_back(i);
    if (which.empty()) continue;
    const std::string key = dev + "|wr|" + std::to_string(c);
    int opts[4];
    const int no = ragged_wr_options(c, opts);
    if (cache.count(key)) {
      r->wr[c] = cache[key];
      continue;
    }
    const int cov = kRouteCov;
    const ItemList items = make_items(*r, which, &cov, /*force_wg=*/true);
    float best = 1e30f;
    int best_wr = r->wr[c];
    for (int o = 0; e == hipSuccess && o < no; ++o) {
      r->wr[c] = opts[o];
      float ms = 0.f;
      e = time_subset(*r, items, repeats, &ms);
      if (ms < best) {
        best = ms;
        best_wr = opts[o];
      }
    }
    r->wr[c] = best_wr;
    cache[key] = best_wr;
  }
  // 2. small classes: one trial per wave (packed) or per workgroup; the probe
  // holds up to 4 * kRaggedPackWaves * max_probe trials, so that both layouts
  // fill as many workgroups and a packed workgroup gets several tickets (in a
  // single round it would wait for the longest of its eight trials)
  for (int c = 0; e == hipSuccess && c < kRaggedPackClasses; ++c) {
    if (r->plan->shape1 != 1) break;  // the packed path needs a 1-D grid
    std::vector<size_t> which;
    for (size_t i = 0; i < n && int(which.size()) < 4 * kRaggedPackWaves * max_probe; ++i)
      if (r->cls[i] == c) which.push_back(i);
    if (which.empty()) continue;
    const std::string key = dev + "|pack|" + std::to_string(c);
    if (cache.count(key)) {
      r->pack[c] = cache[key] != 0;
      continue;
    }
    const int cov = kRouteCov;
    float t[2] = {0.f, 0.f};
    for (int pk = 0; e == hipSuccess && pk < 2; ++pk) {
      r->pack[c] = pk != 0;
      e = time_subset(*r, make_items(*r, which, &cov), repeats, &t[pk]);
    }
    r->pack[c] = t[1] < t[0];
    cache[key] = r->pack[c] ? 1 : 0;
  }
  // 3. routes per (size class, snapshot-count bucket) where both routes exist
  for (int c = 0; e == hipSuccess && c < kRaggedClasses; ++c) {
    std::map<int, std::vector<size_t>> buckets;
    for (size_t i = 0; i < n; ++i)
      if (r->cls[i] == c && r->desc[i].route == BA_ROUTE_AUTO && snapshot_allowed(r->desc[i].n_snap, c) &&
          int(buckets[bucket_of(r->desc[i].n_snap)].size()) < max_probe)
        buckets[bucket_of(r->desc[i].n_snap)].push_back(i);
    for (auto& kv : buckets) {
      const std::string key = dev + "|route|" + std::to_string(c) + "|" + std::to_string(kv.first);
      if (cache.count(key)) {
        r->route_table[{c, kv.first}] = cache[key];
        continue;
      }
      float t[2] = {0.f, 0.f};
      for (int rt = 0; e == hipSuccess && rt < 2; ++rt) e = time_subset(*r, make_items(*r, kv.second, &rt), repeats, &t[rt]);
      const int best = t[1] < t[0] ? kRouteSnap : kRouteCov;
      r->route_table[{c, kv.first}] = best;
      cache[key] = best;
    }
  }
  if (e == hipSuccess) {
    std::vector<size_t> all(n);
    for (size_t i = 0; i < n; ++i) all[i] = i;
    e = upload_items(*r, make_items(*r, all, nullptr));
  }
  if (e == hipSuccess) e = capture(*r);
  (void)hipSetDevice(cur);
  if (e != hipSuccess) return rg_dev(fn, e);
  if (cache_path) {
    std::ofstream o(cache_path);
    for (auto& kv : cache) o << kv.first << " " << kv.second << "\n";
  }
  return BA_OK;
}

ba_status ba_ragged_config(ba_ragged r, int32_t* wr_per_class) {
  if (!r || !wr_per_class) return rg_arg("ba_ragged_config", "null argument");
  for (int c = 0; c < kRaggedClasses; ++c) wr_per_class[c] = r->wr[c];
  return BA_OK;
}

ba_status ba_ragged_packed(ba_ragged r, int32_t* packed_per_class) {
  if (!r || !packed_per_class) return rg_arg("ba_ragged_packed", "null argument");
  for (int c = 0; c < kRaggedClasses; ++c)
    packed_per_class[c] = (c < kRaggedPackClasses && r->pack[c] && r->plan->shape1 == 1) ? 1 : 0;
  return BA_OK;
}

ba_status ba_ragged_destroy(ba_ragged r) {
  if (!r) return BA_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(r->device);
  (void)hipDeviceSynchronize();
  rg_free(r);
  (void)hipSetDevice(cur);
  return BA_OK;
}

}  // extern "C"
