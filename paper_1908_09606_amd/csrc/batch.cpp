// Batches of independent products (Algorithm 1's "for all p_i in parallel"
// over many problems of uneven size) as persistent launches.
//
// Every problem gets a tile from a policy; problems that share a tile form
// one group, whose (problem, tile) work items run in one persistent launch
// with workgroups pulling items from a device counter.  Items are ordered
// longest first (k, then tile count), so the tail of a launch is made of
// short items.  A batch handle captures the launches into a HIP graph.
//
// Autotuner: candidate policies are the planner's per-problem choice (its
// time / I/O model, split factor fixed to 1 inside a batch) and a few
// uniform and size-threshold assignments; cosma_batch_create times each
// candidate's graph on the real batch and keeps the fastest.  Tuning runs
// the batch, so it is done only when every beta is zero (the outputs are then
// simply overwritten); otherwise the planner's policy is used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/cosma_mi355.h"
#include "kernels.hpp"
#include "planner.hpp"
#include "runtime.hpp"

namespace cosma {

int batched_occupancy_f64(int tile_id);
int batched_occupancy_f32(int tile_id);

bool batched_form_f32(int tile_id);
bool batched_form(int dtype, int tile_id) { return dtype == F64 || batched_form_f32(tile_id); }

int batched_occupancy(int dtype, int tile_id) {
  return dtype == F64 ? batched_occupancy_f64(tile_id) : batched_occupancy_f32(tile_id);
}

namespace {

struct Group {
  int tile_id;
  int64_t begin, count;  // range in the item list
  int grid;
};

struct Scale {
  void* C;
  int64_t ldc, m, n;
  double beta;
};

struct Batch {
  int dtype = F32;
  int policy = 0;
  double policy_ms[8] = {0};
  std::vector<BatchProblem> probs;
  std::vector<int> input_index;  // probs[i] came from input problem input_index[i]
  std::vector<int> tile_of;      // tile id of probs[i] under the kept policy
  int64_t inputs = 0;
  std::vector<Scale> scales;
  BatchProblem* d_probs = nullptr;
  BatchItem* d_items = nullptr;
  unsigned* d_counters = nullptr;
  std::vector<Group> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

constexpr int kPolicies = 4;

bool autotune_enabled() {
  static bool on = [] {
    const char* e = std::getenv("COSMA_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Tile of problem p under a policy.
int policy_tile(int policy, int dtype, const BatchProblem& p, const cosma_device_facts& f) {
  switch (policy) {
    case 0: {
      // the planner's batch model: padded work at the tile's issue rate
      // against its counted I/O; the cheapest tile wins
      int cnt = 0;
      tile_menu(dtype, &cnt);
      int best = 0;
      double best_t = INFINITY;
      for (int id = 0; id < cnt; ++id) {
        if (!batched_form(dtype, id)) continue;
        const double t = batch_item_cost(p.m, p.n, p.k, dtype, id, f);
        if (t < best_t) {
          best_t = t;
          best = id;
        }
      }
      return best;
    }
    case 1: return 1;                                           // all 64 x 64
    case 2: return 0;                                           // all 128 x 128
    default: return (p.m * p.n >= 1024LL * 1024) ? 0 : 1;      // size threshold
  }
}

// Build groups + items for a policy.
void build_items(Batch& b, int policy, const cosma_device_facts& f, std::vector<BatchItem>& items,
                 std::vector<Group>& groups, std::vector<BatchProblem>& probs) {
  int cnt = 0;
  const TileDesc* menu = tile_menu(b.dtype, &cnt);
  std::vector<std::vector<int>> by_tile(cnt);
  probs = b.probs;
  b.tile_of.assign(probs.size(), 0);
  for (size_t i = 0; i < probs.size(); ++i) {
    const int t = policy_tile(policy, b.dtype, probs[i], f);
    b.tile_of[i] = t;
    probs[i].tiles_m = ceil_div(probs[i].m, menu[t].tm);
    probs[i].tiles_n = ceil_div(probs[i].n, menu[t].tn);
    by_tile[t].push_back((int)i);
  }
  items.clear();
  groups.clear();
  for (int t = 0; t < cnt; ++t) {
    if (by_tile[t].empty()) continue;
    std::vector<int>& ps = by_tile[t];
    // longest items first: k (rounds per item) decides an item's duration
    std::stable_sort(ps.begin(), ps.end(),
                     [&](int a, int c) { return probs[a].k > probs[c].k; });
    Group g;
    g.tile_id = t;
    g.begin = (int64_t)items.size();
    for (int pi : ps) {
      const int64_t tiles = probs[pi].tiles_m * probs[pi].tiles_n;
      for (int64_t q = 0; q < tiles; ++q) items.push_back(BatchItem{pi, (int32_t)q});
    }
    g.count = (int64_t)items.size() - g.begin;
    const int occ = batched_occupancy(b.dtype, t);
    const int64_t slots = (int64_t)f.num_cus * occ;
    g.grid = (int)std::max<int64_t>(1, std::min<int64_t>(slots, g.count));
    groups.push_back(g);
  }
}

int enqueue(const Batch& b, const std::vector<Group>& groups, hipStream_t s) {
  hipError_t e = launch_reset_counters(b.d_counters, (int)groups.size(), s);
  if (e != hipSuccess) return COSMA_ERR_HIP;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    BatchArgs a;
    a.probs = b.d_probs;
    a.items = b.d_items + g.begin;
    a.count = g.count;
    a.counter = b.d_counters + gi;
    e = b.dtype == F64 ? launch_batched_f64(g.tile_id, a, g.grid, s)
                       : launch_batched_f32(g.tile_id, a, g.grid, s);
    if (e != hipSuccess) return COSMA_ERR_HIP;
  }
  for (const Scale& sc : b.scales) {
    e = b.dtype == F64 ? launch_scale_f64((double*)sc.C, sc.ldc, sc.m, sc.n, sc.beta, s)
                       : launch_scale_f32((float*)sc.C, sc.ldc, sc.m, sc.n, (float)sc.beta, s);
    if (e != hipSuccess) return COSMA_ERR_HIP;
  }
  return COSMA_OK;
}

void free_device(Batch& b) {
  if (b.exec) hipGraphExecDestroy(b.exec);
  if (b.graph) hipGraphDestroy(b.graph);
  if (b.d_probs) hipFree(b.d_probs);
  if (b.d_items) hipFree(b.d_items);
  if (b.d_counters) hipFree(b.d_counters);
  b.exec = nullptr;
  b.graph = nullptr;
  b.d_probs = nullptr;
  b.d_items = nullptr;
  b.d_counters = nullptr;
}

// Upload a policy's lists and capture its graph (on a private stream).
int materialise(Batch& b, int policy, const cosma_device_facts& f) {
  std::vector<BatchItem> items;
  std::vector<Group> groups;
  std::vector<BatchProblem> probs;
  build_items(b, policy, f, items, groups, probs);
  free_device(b);
  const size_t pb = std::max<size_t>(1, probs.size()) * sizeof(BatchProblem);
  const size_t ib = std::max<size_t>(1, items.size()) * sizeof(BatchItem);
  if (hipMalloc(&b.d_probs, pb) != hipSuccess || hipMalloc(&b.d_items, ib) != hipSuccess ||
      hipMalloc(&b.d_counters, 64 * sizeof(unsigned)) != hipSuccess) {
    free_device(b);
    return COSMA_ERR_HIP;
  }
  if (!probs.empty() &&
      hipMemcpy(b.d_probs, probs.data(), probs.size() * sizeof(BatchProblem),
                hipMemcpyHostToDevice) != hipSuccess)
    return COSMA_ERR_HIP;
  if (!items.empty() &&
      hipMemcpy(b.d_items, items.data(), items.size() * sizeof(BatchItem),
                hipMemcpyHostToDevice) != hipSuccess)
    return COSMA_ERR_HIP;
  b.groups = groups;
  b.policy = policy;
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return COSMA_ERR_HIP;
  int rc = COSMA_OK;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = COSMA_ERR_HIP;
  } else {
    rc = enqueue(b, b.groups, cap);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(cap, &g);
    if (rc == COSMA_OK && ee == hipSuccess) {
      b.graph = g;
      if (hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0) != hipSuccess) rc = COSMA_ERR_HIP;
    } else {
      if (g) hipGraphDestroy(g);
      rc = COSMA_ERR_HIP;
    }
  }
  hipStreamDestroy(cap);
  return rc;
}

// Time a materialised batch: one warm replay, then the median of three.
double time_graph(Batch& b, hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e300;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return 1e300;
  }
  double ts[3] = {1e300, 1e300, 1e300};
  if (hipGraphLaunch(b.exec, s) == hipSuccess) {
    for (int r = 0; r < 3; ++r) {
      hipEventRecord(e0, s);
      hipGraphLaunch(b.exec, s);
      hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) == hipSuccess) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        ts[r] = ms;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  std::sort(ts, ts + 3);
  return ts[1];
}

int check_problem(int64_t m, int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
                  const void* B, int64_t ldb, const void* C, int64_t ldc, size_t el) {
  if (m < 0 || n < 0 || k < 0) return COSMA_ERR_INVALID_ARG;
  if (lda < std::max<int64_t>(1, k) || ldb < std::max<int64_t>(1, n) || ldc < std::max<int64_t>(1, n))
    return COSMA_ERR_INVALID_ARG;
  if (m == 0 || n == 0) return COSMA_OK;
  if (!C || (uintptr_t)C % el) return COSMA_ERR_INVALID_ARG;
  if (k > 0 && alpha != 0.0 && (!A || !B || (uintptr_t)A % el || (uintptr_t)B % el))
    return COSMA_ERR_INVALID_ARG;
  if (m > (1LL << 30) || n > (1LL << 30)) return COSMA_ERR_UNSUPPORTED;
  return COSMA_OK;
}

int collect(Batch& b, int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
            const double* alpha, const void* const* A, const int64_t* lda, const void* const* B,
            const int64_t* ldb, const double* beta, void* const* C, const int64_t* ldc, int dtype) {
  if (count < 0 || (count > 0 && (!m || !n || !k || !alpha || !A || !lda || !B || !ldb || !beta ||
                                  !C || !ldc)))
    return COSMA_ERR_INVALID_ARG;
  if (dtype != F32 && dtype != F64) return COSMA_ERR_UNSUPPORTED;
  if (count > (1LL << 24)) return COSMA_ERR_UNSUPPORTED;
  b.dtype = dtype;
  b.inputs = count;
  const size_t el = (size_t)word_bytes(dtype);
  int64_t total_items = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int rc = check_problem(m[i], n[i], k[i], alpha[i], A[i], lda[i], B[i], ldb[i], C[i],
                                 ldc[i], el);
    if (rc != COSMA_OK) return rc;
    if (m[i] == 0 || n[i] == 0) continue;
    if (k[i] == 0 || alpha[i] == 0.0) {
      b.scales.push_back(Scale{C[i], ldc[i], m[i], n[i], beta[i]});
      continue;
    }
    BatchProblem p;
    std::memset(&p, 0, sizeof(p));
    p.A = A[i];
    p.B = B[i];
    p.C = C[i];
    p.lda = lda[i];
    p.ldb = ldb[i];
    p.ldc = ldc[i];
    p.m = m[i];
    p.n = n[i];
    p.k = k[i];
    p.alpha = alpha[i];
    p.beta = beta[i];
    p.vec_a = ((uintptr_t)A[i] % 16 == 0 && ((size_t)lda[i] * el) % 16 == 0) ? 1 : 0;
    p.vec_b = ((uintptr_t)B[i] % 16 == 0 && ((size_t)ldb[i] * el) % 16 == 0) ? 1 : 0;
    b.probs.push_back(p);
    b.input_index.push_back((int)i);
    total_items += ceil_div(m[i], 64) * ceil_div(n[i], 64);
    if (total_items > 0x7fffffffLL) return COSMA_ERR_UNSUPPORTED;
  }
  return COSMA_OK;
}

}  // namespace
}  // namespace cosma

using namespace cosma;

extern "C" {

int cosma_batch_create(int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* alpha, const void* const* A, const int64_t* lda,
                       const void* const* B, const int64_t* ldb, const double* beta,
                       void* const* C, const int64_t* ldc, int dtype, void* stream,
                       void** handle) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  *handle = nullptr;
  Batch* b = new (std::nothrow) Batch();
  if (!b) return COSMA_ERR_NO_MEMORY;
  int rc = collect(*b, count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
  if (rc == COSMA_OK) {
    int st = COSMA_OK;
    const cosma_device_facts f = device_facts(&st);
    rc = st;
    if (rc == COSMA_OK) {
      bool all_beta_zero = true;
      for (const BatchProblem& p : b->probs) all_beta_zero = all_beta_zero && p.beta == 0.0;
      for (const auto& s : b->scales) all_beta_zero = all_beta_zero && s.beta == 0.0;
      int best = 0;
      if (autotune_enabled() && all_beta_zero && !b->probs.empty()) {
        double best_ms = 1e300;
        for (int pol = 0; pol < kPolicies && rc == COSMA_OK; ++pol) {
          rc = materialise(*b, pol, f);
          if (rc != COSMA_OK) break;
          const double ms = time_graph(*b, (hipStream_t)stream);
          b->policy_ms[pol] = ms;
          if (ms < best_ms) {
            best_ms = ms;
            best = pol;
          }
        }
      }
      if (rc == COSMA_OK) rc = materialise(*b, best, f);
    }
  }
  if (rc != COSMA_OK) {
    free_device(*b);
    delete b;
    return rc;
  }
  *handle = b;
  return COSMA_OK;
}

int cosma_batch_run(void* handle, void* stream) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (!b->exec) return COSMA_ERR_INVALID_ARG;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? COSMA_OK : COSMA_ERR_HIP;
}

int cosma_batch_destroy(void* handle) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  // the graph may still be running: wait for the device before freeing
  hipDeviceSynchronize();
  free_device(*b);
  delete b;
  return COSMA_OK;
}

int cosma_batch_info(void* handle, int* policy, int* groups, int64_t* items, double* policy_ms,
                     int policy_ms_len) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (policy) *policy = b->policy;
  if (groups) *groups = (int)b->groups.size();
  if (items) {
    int64_t t = 0;
    for (const Group& g : b->groups) t += g.count;
    *items = t;
  }
  for (int i = 0; policy_ms && i < policy_ms_len && i < kPolicies; ++i) policy_ms[i] = b->policy_ms[i];
  return COSMA_OK;
}

int cosma_batch_tiles(void* handle, int64_t count, int32_t* tile_ids) {
  if (!handle || !tile_ids) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (count != b->inputs) return COSMA_ERR_INVALID_ARG;
  for (int64_t i = 0; i < count; ++i) tile_ids[i] = -1;
  for (size_t i = 0; i < b->probs.size() && i < b->tile_of.size(); ++i)
    tile_ids[b->input_index[i]] = b->tile_of[i];
  return COSMA_OK;
}

// One-shot batch: the planner's policy, launched directly on `stream`.  The
// work list lives in device memory owned by the library for this device,
// grown on demand and reused; consecutive calls are ordered after each other
// through an event, so calls on different streams do not race on it.
int cosma_gemm_batched(int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* alpha, const void* const* A, const int64_t* lda,
                       const void* const* B, const int64_t* ldb, const double* beta,
                       void* const* C, const int64_t* ldc, int dtype, void* stream) {
  Batch b;
  int rc = collect(b, count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
  if (rc != COSMA_OK) return rc;
  int st = COSMA_OK;
  const cosma_device_facts f = device_facts(&st);
  if (st != COSMA_OK) return st;
  std::vector<BatchItem> items;
  std::vector<Group> groups;
  std::vector<BatchProblem> probs;
  build_items(b, 0, f, items, groups, probs);

  static std::mutex mu;
  static struct Cache {
    BatchProblem* probs = nullptr;
    size_t probs_cap = 0;
    BatchItem* items = nullptr;
    size_t items_cap = 0;
    unsigned* counters = nullptr;
    hipEvent_t done = nullptr;
    int device = -1;
  } cache[64];
  const int dev = current_device();
  if (dev < 0 || dev >= 64) return COSMA_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(mu);
  Cache& c = cache[dev];
  hipStream_t s = (hipStream_t)stream;
  if (c.done && hipStreamWaitEvent(s, c.done, 0) != hipSuccess) return COSMA_ERR_HIP;
  auto grow = [&](void** p, size_t* cap, size_t need) -> bool {
    if (*cap >= need) return true;
    if (*p) {
      if (hipDeviceSynchronize() != hipSuccess) return false;
      hipFree(*p);
      *p = nullptr;
      *cap = 0;
    }
    size_t want = std::max(need, (size_t)4096);
    if (hipMalloc(p, want) != hipSuccess) return false;
    *cap = want;
    return true;
  };
  if (!grow((void**)&c.probs, &c.probs_cap, probs.size() * sizeof(BatchProblem) + 64) ||
      !grow((void**)&c.items, &c.items_cap, items.size() * sizeof(BatchItem) + 64))
    return COSMA_ERR_HIP;
  if (!c.counters && hipMalloc(&c.counters, 64 * sizeof(unsigned)) != hipSuccess) return COSMA_ERR_HIP;
  if (!c.done && hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess)
    return COSMA_ERR_HIP;
  if (groups.size() > 64) return COSMA_ERR_UNSUPPORTED;
  if (!probs.empty() && hipMemcpyAsync(c.probs, probs.data(), probs.size() * sizeof(BatchProblem),
                                       hipMemcpyHostToDevice, s) != hipSuccess)
    return COSMA_ERR_HIP;
  if (!items.empty() && hipMemcpyAsync(c.items, items.data(), items.size() * sizeof(BatchItem),
                                       hipMemcpyHostToDevice, s) != hipSuccess)
    return COSMA_ERR_HIP;
  // the host vectors are released on return: make sure the copies have read them
  if (hipStreamSynchronize(s) != hipSuccess) return COSMA_ERR_HIP;
  b.d_probs = c.probs;
  b.d_items = c.items;
  b.d_counters = c.counters;
  rc = enqueue(b, groups, s);
  b.d_probs = nullptr;
  b.d_items = nullptr;
  b.d_counters = nullptr;
  if (rc != COSMA_OK) return rc;
  return hipEventRecord(c.done, s) == hipSuccess ? COSMA_OK : COSMA_ERR_HIP;
}

}  // extern "C"
