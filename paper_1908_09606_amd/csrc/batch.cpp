// Batches of independent products (Algorithm 1's "for all p_i in parallel"
// over many problems of uneven size) as persistent launches.
//
// Every problem gets a tile and a split factor p_k from a policy; problems
// that share a tile form one group, whose (problem, split, tile) work items
// run in one persistent launch with workgroups pulling items from device
// counters, one per XCD chunk of the group's problems (a problem's panels
// then meet in one L2).  Within a chunk problems are ordered longest item
// first, so the tail of a launch is made of short items.  A problem whose items would be long against the
// launch's share of work per resident slot is cut in k: the batch analogue
// of section 6.2, where k is cut once the processors outnumber the
// independent (i, j) domains.  Its partials go to workspace planes and one
// batched reduction per batch adds them (Reduce).
//
// Two ways to run a batch:
//  - cosma_gemm_batched: one-shot.  Descriptors, the item map, counters and
//    partials live in the caller's registered workspace; descriptors reach
//    it inside kernel arguments, so the call allocates nothing, copies
//    nothing from the host, never waits, and can be captured into a graph.
//  - cosma_batch_create / run: the handle owns device memory (allocated at
//    creation) and a HIP graph of the launches.  The autotuner times
//    candidate policies on the real batch and keeps the fastest; tuning runs
//    the batch, so it is done only when every beta is zero (outputs are then
//    simply overwritten); otherwise the planner's policy is used.
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

// Policies: how each problem gets its tile (and whether it may be split).
enum Policy {
  POLICY_MODEL = 0,      // the planner's batch cost model per problem, splits by the model
  POLICY_ALL_64 = 1,     // every problem on 64 x 64, splits by the model
  POLICY_ALL_128 = 2,    // every problem on 128 x 128, splits by the model
  POLICY_THRESHOLD = 3,  // 128 x 128 from m n >= 2^20, else 64 x 64, splits by the model
  POLICY_NO_SPLIT = 4,   // the model's tiles, k never cut
  POLICY_ONE_TILE = 5,   // one tile for the whole batch: the lowest summed model cost, model splits
  kPolicies = 6
};
// What the one-shot call and an untuned handle use: one persistent launch
// (tile groups run one after another on a stream, so several groups pay
// several launch tails), on the tile whose modelled item costs sum lowest.
constexpr int kDefaultPolicy = POLICY_ONE_TILE;

// A problem as given, before a policy is applied.
struct Input {
  BatchProblem p;  // tiles / split fields filled by the policy
  int index;       // position in the caller's arrays
};

struct Scale {
  void* C;
  int64_t ldc, m, n;
  double beta;
};

struct Group {
  int tile_id;
  int64_t base, items;  // batch-wide item range
  int grid;
  int chunks;                       // XCD chunks (BatchArgs)
  int64_t chunk[kBatchChunks + 1];  // chunk boundaries, launch-relative
};

// A batch under one policy: problems in launch order, groups, reduction list.
struct Layout {
  std::vector<BatchProblem> probs;
  std::vector<int> input_of;   // probs[i] came from input problem input_of[i]
  std::vector<int> in_pos;     // ... at position in_pos[i] of the collected inputs
  std::vector<Group> groups;
  std::vector<int32_t> reduce;  // probs indices with splits > 1
  int64_t items = 0;
  int64_t max_reduce_elems = 0;
  size_t partial_bytes = 0;     // all partial planes, each 256-byte aligned
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

bool autotune_enabled() {
  static bool on = [] {
    const char* e = std::getenv("COSMA_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

int policy_tile(int policy, int dtype, const BatchProblem& p, const cosma_device_facts& f) {
  switch (policy) {
    case POLICY_ALL_64: return 1;
    case POLICY_ALL_128: return 0;
    case POLICY_THRESHOLD: return (p.m * p.n >= 1024LL * 1024) ? 0 : 1;
    default: {
      // padded work at the tile's issue rate against its counted I/O; the
      // cheapest tile with a batched form wins
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
  }
}

// Split factors of one group.  An item runs its whole k range on one
// resident slot, so the launch cannot end before its longest item; with
// items started longest first, a launch is balanced while no item exceeds
// a quarter of the group's work per slot.  Longer items are cut in k (at
// least 256 per split, at most 64 splits), as make_plan cuts k into
// multiples of the tile's round.  req[i] > 0 asks for that many splits of
// group[i] instead (within the same limits).
void choose_splits(std::vector<BatchProblem*>& group, const std::vector<int>& req_in, int dtype,
                   int tile_id, const cosma_device_facts& f) {
  int cnt = 0;
  const TileDesc* menu = tile_menu(dtype, &cnt);
  const TileDesc& T = menu[tile_id];
  const double slots = (double)f.num_cus * (double)batched_occupancy(dtype, tile_id);
  const double slot_rate =
      useful_flops_per_clk_per_cu(dtype, 0) * f.clock_ghz * 1e9 * T.eff * (double)f.num_cus / slots;
  double work = 0.0;  // item-seconds
  for (BatchProblem* p : group)
    work += (double)p->tiles_m * p->tiles_n * 2.0 * T.tm * T.tn * (double)p->k / slot_rate;
  const double cap = work / slots / 4.0;
  for (size_t i = 0; i < group.size(); ++i) {
    BatchProblem* p = group[i];
    const int64_t panels = ceil_div(p->k, T.tk);
    int64_t req = req_in[i];
    if (req <= 0) {
      req = 1;
      const double d = 2.0 * T.tm * T.tn * (double)p->k / slot_rate;
      if (cap > 0.0 && d > cap) req = (int64_t)std::ceil(d / cap);
    }
    req = std::min<int64_t>(req, std::min<int64_t>(64, p->k / 256));
    req = std::max<int64_t>(req, 1);
    p->k_split = ceil_div(panels, req) * T.tk;
    p->splits = (int32_t)ceil_div(p->k, p->k_split);
  }
}

// Tile and split request of every input problem (split 0: the group's
// model, choose_splits).  A policy gives the first assignment; the
// autotuner changes it class by class.
struct Assignment {
  std::vector<int> tile, split;
};

Assignment seed_assignment(const std::vector<Input>& in, int dtype, int policy,
                           const cosma_device_facts& f) {
  Assignment a;
  a.tile.resize(in.size());
  a.split.assign(in.size(), policy == POLICY_NO_SPLIT ? 1 : 0);
  if (policy == POLICY_ONE_TILE) {
    int cnt = 0;
    tile_menu(dtype, &cnt);
    int best = 0;
    double best_t = INFINITY;
    for (int id = 0; id < cnt; ++id) {
      if (!batched_form(dtype, id)) continue;
      double t = 0.0;
      for (const Input& q : in) t += batch_item_cost(q.p.m, q.p.n, q.p.k, dtype, id, f);
      if (t < best_t) {
        best_t = t;
        best = id;
      }
    }
    a.tile.assign(in.size(), best);
    return a;
  }
  for (size_t i = 0; i < in.size(); ++i) a.tile[i] = policy_tile(policy, dtype, in[i].p, f);
  return a;
}

// Apply an assignment: tiles, splits, launch order, item numbering, partials.
void build_layout(const std::vector<Input>& in, int dtype, const Assignment& as,
                  const cosma_device_facts& f, Layout& L) {
  int cnt = 0;
  const TileDesc* menu = tile_menu(dtype, &cnt);
  std::vector<std::vector<int>> by_tile(cnt);
  std::vector<BatchProblem> work(in.size());
  for (size_t i = 0; i < in.size(); ++i) {
    work[i] = in[i].p;
    const int t = as.tile[i];
    work[i].tiles_m = (int32_t)ceil_div(work[i].m, menu[t].tm);
    work[i].tiles_n = (int32_t)ceil_div(work[i].n, menu[t].tn);
    by_tile[t].push_back((int)i);
  }
  L = Layout();
  for (int t = 0; t < cnt; ++t) {
    if (by_tile[t].empty()) continue;
    std::vector<BatchProblem*> group;
    std::vector<int> req;
    for (int i : by_tile[t]) {
      group.push_back(&work[i]);
      req.push_back(as.split[i]);
    }
    choose_splits(group, req, dtype, t, f);
    // One chunk per XCD: whole problems, largest first, each to the chunk
    // with the least work so far; inside a chunk longest items first (the
    // rounds per item decide an item's duration).
    std::vector<int>& ps = by_tile[t];
    auto rounds = [&](int i) {
      const BatchProblem& p = work[i];
      return (double)p.tiles_m * p.tiles_n * p.splits * (double)p.k_split;
    };
    std::stable_sort(ps.begin(), ps.end(), [&](int a, int c) { return rounds(a) > rounds(c); });
    Group g;
    g.tile_id = t;
    g.base = L.items;
    g.chunks = std::max(1, std::min(kBatchChunks, f.num_xcds));
    std::vector<std::vector<int>> bins(g.chunks);
    std::vector<double> load(g.chunks, 0.0);
    for (int i : ps) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      bins[x].push_back(i);
      load[x] += rounds(i);
    }
    for (int x = 0; x < g.chunks; ++x) {
      std::stable_sort(bins[x].begin(), bins[x].end(),
                       [&](int a, int c) { return work[a].k_split > work[c].k_split; });
      g.chunk[x] = L.items - g.base;
      for (int i : bins[x]) {
        BatchProblem p = work[i];
        p.first = L.items;
        L.items += (int64_t)p.tiles_m * p.tiles_n * p.splits;
        L.input_of.push_back(in[i].index);
        L.in_pos.push_back(i);
        L.probs.push_back(p);
      }
    }
    g.items = L.items - g.base;
    for (int x = g.chunks; x <= kBatchChunks; ++x) g.chunk[x] = g.items;
    const int64_t slots = (int64_t)f.num_cus * batched_occupancy(dtype, t);
    g.grid = (int)std::max<int64_t>(1, std::min<int64_t>(slots, g.items));
    L.groups.push_back(g);
  }
  const size_t w = (size_t)word_bytes(dtype);
  for (size_t i = 0; i < L.probs.size(); ++i) {
    BatchProblem& p = L.probs[i];
    if (p.splits <= 1) continue;
    p.P = reinterpret_cast<void*>(L.partial_bytes);  // offset until placed
    L.partial_bytes += up256((size_t)p.splits * (size_t)p.m * (size_t)p.n * w);
    L.reduce.push_back((int32_t)i);
    L.max_reduce_elems = std::max<int64_t>(L.max_reduce_elems, p.m * p.n);
  }
}

// Device memory a layout needs: descriptors, item map, counters, partials.
struct DeviceParts {
  size_t probs, map, counters, partials, total;
};

DeviceParts parts_of(const Layout& L) {
  DeviceParts d;
  d.probs = up256(std::max<size_t>(1, L.probs.size()) * sizeof(BatchProblem));
  d.map = up256(std::max<int64_t>(1, L.items) * sizeof(int32_t));
  d.counters = up256(std::max<size_t>(1, L.groups.size()) * kBatchChunks * sizeof(unsigned));
  d.partials = L.partial_bytes;
  d.total = d.probs + d.map + d.counters + d.partials;
  return d;
}

// Pointers of a layout placed at `base` (device memory of parts_of(L).total
// bytes, 256-byte aligned): partial offsets become addresses.
struct Placed {
  BatchProblem* probs;
  int32_t* map;
  unsigned* counters;
  char* partials;
};

Placed place(Layout& L, void* base) {
  const DeviceParts d = parts_of(L);
  Placed pl;
  char* b = static_cast<char*>(base);
  pl.probs = reinterpret_cast<BatchProblem*>(b);
  pl.map = reinterpret_cast<int32_t*>(b + d.probs);
  pl.counters = reinterpret_cast<unsigned*>(b + d.probs + d.map);
  pl.partials = b + d.probs + d.map + d.counters;
  for (BatchProblem& p : L.probs)
    if (p.splits > 1) p.P = pl.partials + reinterpret_cast<uintptr_t>(p.P);
  return pl;
}

// Everything after the descriptors are in device memory: the item map,
// counters, one persistent launch per group, the reduction, beta scaling of
// problems without products.  Kernel launches only (graph-capture safe).
// With `side` (a fork event, and a stream and a join event per group after
// the first; used while capturing) the groups' launches fork from `s` and join it again
// before the reduction, so a group's workgroups take the CUs that the
// previous group's last items leave idle.
struct SideStreams {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> fork, join;
};

int enqueue_launches(int dtype, const Layout& L, const Placed& pl, const std::vector<Scale>& scales,
                     hipStream_t s, const SideStreams* side = nullptr) {
  if (!L.probs.empty()) {
    if (launch_batch_expand(pl.probs, (int64_t)L.probs.size(), pl.map, s) != hipSuccess)
      return COSMA_ERR_HIP;
    if (launch_reset_counters(pl.counters, (int)L.groups.size() * kBatchChunks, s) != hipSuccess)
      return COSMA_ERR_HIP;
  }
  // one fork point after the map and counters, before any group's launch
  const bool fork = side && L.groups.size() > 1 && side->streams.size() + 1 >= L.groups.size();
  if (fork && hipEventRecord(side->fork[0], s) != hipSuccess) return COSMA_ERR_HIP;
  for (size_t gi = 0; gi < L.groups.size(); ++gi) {
    const Group& g = L.groups[gi];
    hipStream_t gs = s;
    if (fork && gi > 0) {
      gs = side->streams[gi - 1];
      if (hipStreamWaitEvent(gs, side->fork[0], 0) != hipSuccess) return COSMA_ERR_HIP;
    }
    BatchArgs a;
    a.probs = pl.probs;
    a.map = pl.map;
    a.base = g.base;
    a.count = g.items;
    a.counter = pl.counters + gi * kBatchChunks;
    a.chunks = g.chunks;
    a.pad_ = 0;
    for (int x = 0; x <= kBatchChunks; ++x) a.chunk[x] = g.chunk[x];
    const hipError_t e = dtype == F64 ? launch_batched_f64(g.tile_id, a, g.grid, gs)
                                      : launch_batched_f32(g.tile_id, a, g.grid, gs);
    if (e != hipSuccess) return COSMA_ERR_HIP;
  }
  if (fork)
    for (size_t gi = 1; gi < L.groups.size(); ++gi)
      if (hipEventRecord(side->join[gi - 1], side->streams[gi - 1]) != hipSuccess ||
          hipStreamWaitEvent(s, side->join[gi - 1], 0) != hipSuccess)
        return COSMA_ERR_HIP;
  for (size_t r0 = 0; r0 < L.reduce.size(); r0 += kReduceList) {
    BatchReduceArgs r;
    r.probs = pl.probs;
    r.count = (int32_t)std::min<size_t>(kReduceList, L.reduce.size() - r0);
    for (int i = 0; i < r.count; ++i) r.idx[i] = L.reduce[r0 + i];
    if (launch_batch_reduce(dtype, r, L.max_reduce_elems, s) != hipSuccess) return COSMA_ERR_HIP;
  }
  for (const Scale& sc : scales) {
    const hipError_t e =
        dtype == F64 ? launch_scale_f64((double*)sc.C, sc.ldc, sc.m, sc.n, sc.beta, s)
                     : launch_scale_f32((float*)sc.C, sc.ldc, sc.m, sc.n, (float)sc.beta, s);
    if (e != hipSuccess) return COSMA_ERR_HIP;
  }
  return COSMA_OK;
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

// Validate the caller's arrays and split them into problems with products
// and beta-only scalings.  Pointers may be null when only sizes matter
// (workspace queries: with_pointers = false).
int collect(int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
            const double* alpha, const void* const* A, const int64_t* lda, const void* const* B,
            const int64_t* ldb, const double* beta, void* const* C, const int64_t* ldc, int dtype,
            bool with_pointers, std::vector<Input>& in, std::vector<Scale>& scales) {
  if (count < 0 || (count > 0 && (!m || !n || !k || !alpha)))
    return COSMA_ERR_INVALID_ARG;
  if (with_pointers && count > 0 && (!A || !lda || !B || !ldb || !beta || !C || !ldc))
    return COSMA_ERR_INVALID_ARG;
  if (dtype != F32 && dtype != F64) return COSMA_ERR_UNSUPPORTED;
  if (count > (1LL << 24)) return COSMA_ERR_UNSUPPORTED;
  const size_t el = (size_t)word_bytes(dtype);
  int64_t total_items = 0;
  for (int64_t i = 0; i < count; ++i) {
    if (with_pointers) {
      const int rc = check_problem(m[i], n[i], k[i], alpha[i], A[i], lda[i], B[i], ldb[i], C[i],
                                   ldc[i], el);
      if (rc != COSMA_OK) return rc;
    } else if (m[i] < 0 || n[i] < 0 || k[i] < 0) {
      return COSMA_ERR_INVALID_ARG;
    } else if (m[i] > (1LL << 30) || n[i] > (1LL << 30)) {
      return COSMA_ERR_UNSUPPORTED;
    }
    if (m[i] == 0 || n[i] == 0) continue;
    if (k[i] == 0 || alpha[i] == 0.0) {
      if (with_pointers) scales.push_back(Scale{C[i], ldc[i], m[i], n[i], beta[i]});
      continue;
    }
    Input q;
    std::memset(&q, 0, sizeof(q));
    BatchProblem& p = q.p;
    if (with_pointers) {
      p.A = A[i];
      p.B = B[i];
      p.C = C[i];
      p.lda = lda[i];
      p.ldb = ldb[i];
      p.ldc = ldc[i];
      p.beta = beta[i];
      p.vec_a = ((uintptr_t)A[i] % 16 == 0 && ((size_t)lda[i] * el) % 16 == 0) ? 1 : 0;
      p.vec_b = ((uintptr_t)B[i] % 16 == 0 && ((size_t)ldb[i] * el) % 16 == 0) ? 1 : 0;
    }
    p.m = m[i];
    p.n = n[i];
    p.k = k[i];
    p.alpha = alpha[i];
    q.index = (int)i;
    in.push_back(q);
    // the item map holds int32 problem indices and items (64 x 64 tiles, at
    // most 64 splits each)
    total_items += ceil_div(m[i], 64) * ceil_div(n[i], 64) * 64;
    if (total_items > 0x7fffffffLL) return COSMA_ERR_UNSUPPORTED;
  }
  return COSMA_OK;
}

// ---- batch handles -------------------------------------------------------

struct Batch {
  int dtype = F32;
  int policy = kDefaultPolicy;
  double policy_ms[kPolicies] = {0};
  int trials = 0;         // refinement trials the autotuner timed
  double seed_ms = 0.0;   // best policy's time
  double tuned_ms = 0.0;  // the kept assignment's time
  std::vector<Input> inputs;
  std::vector<Scale> scales;
  int64_t count = 0;
  Layout layout;
  void* mem = nullptr;  // descriptors, map, counters, partials
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // the last replay enqueued outside a capture
  bool recorded = false;
};

void free_device(Batch& b) {
  if (b.exec) hipGraphExecDestroy(b.exec);
  if (b.graph) hipGraphDestroy(b.graph);
  if (b.mem) hipFree(b.mem);
  b.exec = nullptr;
  b.graph = nullptr;
  b.mem = nullptr;
}

void destroy_side(SideStreams& side) {
  for (hipStream_t x : side.streams) hipStreamDestroy(x);
  for (hipEvent_t e : side.fork) hipEventDestroy(e);
  for (hipEvent_t e : side.join) hipEventDestroy(e);
  side = SideStreams();
}

// Lay out an assignment, upload it and capture its launches (private
// streams; the tile groups run concurrently inside the graph).
int materialise(Batch& b, const Assignment& as, const cosma_device_facts& f) {
  free_device(b);
  build_layout(b.inputs, b.dtype, as, f, b.layout);
  const DeviceParts d = parts_of(b.layout);
  if (hipMalloc(&b.mem, d.total) != hipSuccess) {
    b.mem = nullptr;
    return COSMA_ERR_HIP;
  }
  const Placed pl = place(b.layout, b.mem);
  if (!b.layout.probs.empty() &&
      hipMemcpy(pl.probs, b.layout.probs.data(), b.layout.probs.size() * sizeof(BatchProblem),
                hipMemcpyHostToDevice) != hipSuccess)
    return COSMA_ERR_HIP;
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return COSMA_ERR_HIP;
  int rc = COSMA_OK;
  SideStreams side;
  for (size_t gi = 1; gi < b.layout.groups.size() && rc == COSMA_OK; ++gi) {
    hipStream_t x;
    hipEvent_t e;
    if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
      rc = COSMA_ERR_HIP;
      break;
    }
    side.streams.push_back(x);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      rc = COSMA_ERR_HIP;
      break;
    }
    side.join.push_back(e);
    if (side.fork.empty()) {
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        rc = COSMA_ERR_HIP;
        break;
      }
      side.fork.push_back(e);
    }
  }
  if (rc == COSMA_OK && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    rc = COSMA_ERR_HIP;
  if (rc == COSMA_OK) {
    rc = enqueue_launches(b.dtype, b.layout, pl, b.scales, cap, &side);
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
  destroy_side(side);
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

// The splits a layout gave each input, as explicit requests.
Assignment explicit_assignment(const Layout& L, size_t n_inputs) {
  Assignment a;
  a.tile.assign(n_inputs, 0);
  a.split.assign(n_inputs, 1);
  for (const Group& g : L.groups)
    for (size_t i = 0; i < L.probs.size(); ++i)
      if (L.probs[i].first >= g.base && L.probs[i].first < g.base + g.items) {
        a.tile[L.in_pos[i]] = g.tile_id;
        a.split[L.in_pos[i]] = L.probs[i].splits;
      }
  return a;
}

// Autotuner.  Seeds: the policies, each timed on the real batch.  Then,
// starting from the fastest, problems are taken class by class (classes of
// m n and of k, a factor of four wide each, heaviest class first), and each
// class tries the other tiles with a batched form and twice / half its
// current split factors; a change is kept when the batch gets faster by
// more than 1 % (the replay timing's noise).
constexpr int kRefineClasses = 8;
constexpr double kKeepGain = 0.99;

int autotune(Batch& b, const cosma_device_facts& f, hipStream_t s, Assignment& best) {
  int rc = COSMA_OK;
  double best_ms = 1e300;
  for (int pol = 0; pol < kPolicies; ++pol) {
    const Assignment a = seed_assignment(b.inputs, b.dtype, pol, f);
    if ((rc = materialise(b, a, f)) != COSMA_OK) return rc;
    const double ms = time_graph(b, s);
    b.policy_ms[pol] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = explicit_assignment(b.layout, b.inputs.size());
      b.policy = pol;
    }
  }
  b.seed_ms = best_ms;
  // classes by log4(m n) and log4(k), heaviest (sum of 2 m n k) first
  const size_t n_in = b.inputs.size();
  std::vector<int> cls(n_in);
  std::vector<std::pair<double, int>> weight;
  for (size_t i = 0; i < n_in; ++i) {
    const BatchProblem& p = b.inputs[i].p;
    const int cm = (int)std::floor(std::log2((double)p.m * (double)p.n) / 2.0);
    const int ck = (int)std::floor(std::log2((double)p.k) / 2.0);
    cls[i] = cm * 64 + ck;
  }
  for (size_t i = 0; i < n_in; ++i) {
    auto it = std::find_if(weight.begin(), weight.end(),
                           [&](const std::pair<double, int>& w) { return w.second == cls[i]; });
    const BatchProblem& p = b.inputs[i].p;
    const double fl = 2.0 * (double)p.m * (double)p.n * (double)p.k;
    if (it == weight.end())
      weight.emplace_back(fl, cls[i]);
    else
      it->first += fl;
  }
  std::sort(weight.begin(), weight.end(),
            [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
              return x.first > y.first;
            });
  int cnt = 0;
  tile_menu(b.dtype, &cnt);
  for (size_t c = 0; c < weight.size() && (int)c < kRefineClasses; ++c) {
    const int key = weight[c].second;
    std::vector<Assignment> tries;
    for (int t = 0; t < cnt; ++t) {
      if (!batched_form(b.dtype, t)) continue;
      Assignment a = best;
      bool changed = false;
      for (size_t i = 0; i < n_in; ++i)
        if (cls[i] == key && a.tile[i] != t) {
          a.tile[i] = t;
          a.split[i] = 0;  // the model's split for the new tile
          changed = true;
        }
      if (changed) tries.push_back(a);
    }
    for (int dir = 0; dir < 2; ++dir) {
      Assignment a = best;
      bool changed = false;
      for (size_t i = 0; i < n_in; ++i) {
        if (cls[i] != key) continue;
        const int64_t k = b.inputs[i].p.k;
        const int lim = (int)std::max<int64_t>(1, std::min<int64_t>(64, k / 256));
        const int v = dir == 0 ? std::min(lim, a.split[i] * 2) : std::max(1, a.split[i] / 2);
        if (v != a.split[i]) {
          a.split[i] = v;
          changed = true;
        }
      }
      if (changed) tries.push_back(a);
    }
    for (const Assignment& a : tries) {
      if ((rc = materialise(b, a, f)) != COSMA_OK) return rc;
      const double ms = time_graph(b, s);
      ++b.trials;
      if (ms < best_ms * kKeepGain) {
        best_ms = ms;
        best = explicit_assignment(b.layout, n_in);
      }
    }
  }
  b.tuned_ms = best_ms;
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
  b->dtype = dtype;
  b->count = count;
  int rc = collect(count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, true, b->inputs,
                   b->scales);
  if (rc == COSMA_OK) {
    int st = COSMA_OK;
    const cosma_device_facts f = device_facts(&st);
    rc = st;
    if (rc == COSMA_OK && hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess)
      rc = COSMA_ERR_HIP;
    if (rc == COSMA_OK) {
      bool all_beta_zero = true;
      for (const Input& q : b->inputs) all_beta_zero = all_beta_zero && q.p.beta == 0.0;
      for (const Scale& s : b->scales) all_beta_zero = all_beta_zero && s.beta == 0.0;
      Assignment best = seed_assignment(b->inputs, dtype, kDefaultPolicy, f);
      if (autotune_enabled() && all_beta_zero && !b->inputs.empty())
        rc = autotune(*b, f, (hipStream_t)stream, best);
      if (rc == COSMA_OK) rc = materialise(*b, best, f);
    }
  }
  if (rc != COSMA_OK) {
    free_device(*b);
    if (b->done) hipEventDestroy(b->done);
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
  hipStream_t s = (hipStream_t)stream;
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return COSMA_ERR_HIP;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return COSMA_ERR_HIP;
  if (cs == hipStreamCaptureStatusNone) {
    if (hipEventRecord(b->done, s) != hipSuccess) return COSMA_ERR_HIP;
    b->recorded = true;
  }
  return COSMA_OK;
}

int cosma_batch_destroy(void* handle) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  // the last replay may still be running: wait for it (only it) before
  // freeing what it reads
  if (b->recorded) hipEventSynchronize(b->done);
  free_device(*b);
  if (b->done) hipEventDestroy(b->done);
  delete b;
  return COSMA_OK;
}

int cosma_batch_info(void* handle, int* policy, int* groups, int64_t* items, double* policy_ms,
                     int policy_ms_len) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (policy) *policy = b->policy;
  if (groups) *groups = (int)b->layout.groups.size();
  if (items) *items = b->layout.items;
  for (int i = 0; policy_ms && i < policy_ms_len; ++i)
    policy_ms[i] = i < kPolicies ? b->policy_ms[i] : 0.0;
  return COSMA_OK;
}

int cosma_batch_tuning(void* handle, int* trials, double* seed_ms, double* tuned_ms) {
  if (!handle) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (trials) *trials = b->trials;
  if (seed_ms) *seed_ms = b->seed_ms;
  if (tuned_ms) *tuned_ms = b->tuned_ms;
  return COSMA_OK;
}

int cosma_batch_tiles(void* handle, int64_t count, int32_t* tile_ids) {
  if (!handle || !tile_ids) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (count != b->count) return COSMA_ERR_INVALID_ARG;
  for (int64_t i = 0; i < count; ++i) tile_ids[i] = -1;
  for (const Group& g : b->layout.groups)
    for (size_t i = 0; i < b->layout.probs.size(); ++i)
      if (b->layout.probs[i].first >= g.base && b->layout.probs[i].first < g.base + g.items)
        tile_ids[b->layout.input_of[i]] = g.tile_id;
  return COSMA_OK;
}

int cosma_batch_splits(void* handle, int64_t count, int32_t* p_k) {
  if (!handle || !p_k) return COSMA_ERR_INVALID_ARG;
  Batch* b = static_cast<Batch*>(handle);
  if (count != b->count) return COSMA_ERR_INVALID_ARG;
  for (int64_t i = 0; i < count; ++i) p_k[i] = 0;
  for (size_t i = 0; i < b->layout.probs.size(); ++i)
    p_k[b->layout.input_of[i]] = b->layout.probs[i].splits;
  return COSMA_OK;
}

int cosma_workspace_size_batched(int64_t count, const int64_t* m, const int64_t* n,
                                 const int64_t* k, const double* alpha, int dtype, size_t* bytes) {
  if (!bytes) return COSMA_ERR_INVALID_ARG;
  std::vector<Input> in;
  std::vector<Scale> scales;
  int rc = collect(count, m, n, k, alpha, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr, dtype, false, in, scales);
  if (rc != COSMA_OK) return rc;
  int st = COSMA_OK;
  const cosma_device_facts f = device_facts(&st);
  Layout L;
  build_layout(in, dtype, seed_assignment(in, dtype, kDefaultPolicy, f), f, L);
  *bytes = in.empty() ? 0 : parts_of(L).total;
  return COSMA_OK;
}

// One-shot batch under the planner's policy, enqueued on `stream`: the
// descriptors travel inside kernel arguments into the registered workspace,
// which also holds the item map, the counters and the partial planes.
int cosma_gemm_batched(int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* alpha, const void* const* A, const int64_t* lda,
                       const void* const* B, const int64_t* ldb, const double* beta,
                       void* const* C, const int64_t* ldc, int dtype, void* stream) {
  std::vector<Input> in;
  std::vector<Scale> scales;
  int rc = collect(count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, true, in, scales);
  if (rc != COSMA_OK) return rc;
  int st = COSMA_OK;
  const cosma_device_facts f = device_facts(&st);
  if (st != COSMA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Layout L;
  build_layout(in, dtype, seed_assignment(in, dtype, kDefaultPolicy, f), f, L);
  Placed pl{nullptr, nullptr, nullptr, nullptr};
  if (!L.probs.empty()) {
    void* ws = nullptr;
    size_t ws_bytes = 0;
    if (!workspace_for_current(&ws, &ws_bytes) || !ws || ws_bytes < parts_of(L).total)
      return COSMA_ERR_WORKSPACE;
    pl = place(L, ws);
    for (size_t i0 = 0; i0 < L.probs.size(); i0 += kStageProblems) {
      BatchStage stage;
      stage.dst = pl.probs + i0;
      stage.count = (int32_t)std::min<size_t>(kStageProblems, L.probs.size() - i0);
      std::memcpy(stage.p, L.probs.data() + i0, stage.count * sizeof(BatchProblem));
      if (launch_batch_stage(stage, s) != hipSuccess) return COSMA_ERR_HIP;
    }
  }
  return enqueue_launches(dtype, L, pl, scales, s);
}

}  // extern "C"
