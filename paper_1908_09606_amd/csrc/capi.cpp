// C ABI of the library: argument checks, the plan cache, the workspace
// registry and launch sequencing.  See include/cosma_mi355.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cosma_mi355.h"
#include "crt.hpp"
#include "kernels.hpp"
#include "layout.hpp"
#include "ozaki.hpp"
#include "planner.hpp"
#include "runtime.hpp"

namespace cosma {

namespace {

constexpr int kMaxDevices = 64;

struct DeviceState {
  bool queried = false;
  int status = COSMA_OK;  // COSMA_ERR_UNSUPPORTED when not gfx950
  cosma_device_facts facts{};
  void* workspace = nullptr;
  size_t workspace_bytes = 0;
};

std::mutex g_mutex;
DeviceState g_dev[kMaxDevices];
std::map<std::tuple<int, int64_t, int64_t, int64_t, int, int>, cosma_plan_info> g_plans;

double env_delta() {
  static double d = [] {
    const char* e = std::getenv("COSMA_DELTA");
    double v = e ? std::atof(e) : 0.03;
    return (v >= 0.0 && v < 1.0) ? v : 0.03;
  }();
  return d;
}

}  // namespace

// Current device index, or -1 without a usable device.
int current_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return -1;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
  return dev;
}

// Facts of the current device (MI355X defaults when there is none).
// *status: COSMA_OK, or COSMA_ERR_UNSUPPORTED for a device that is not gfx950.
cosma_device_facts device_facts(int* status) {
  const int dev = current_device();
  if (dev < 0) {
    if (status) *status = COSMA_ERR_UNSUPPORTED;
    return mi355x_defaults();
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  DeviceState& d = g_dev[dev];
  if (!d.queried) {
    d.facts = mi355x_defaults();
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) d.status = COSMA_ERR_UNSUPPORTED;
      // the machine model's processor count and fast memory (section 2.1):
      // CUs, and per CU the LDS and the register file (32-bit registers,
      // arch + accumulation); per XCD its L2 and the XCD count for Q_EA.
      // The HBM rate stays the published peak (the clock and bus width the
      // runtime reports do not give it directly).
      if (prop.multiProcessorCount > 0) d.facts.num_cus = prop.multiProcessorCount;
      if (prop.maxSharedMemoryPerMultiProcessor > 0)
        d.facts.lds_bytes_per_cu = (int64_t)prop.maxSharedMemoryPerMultiProcessor;
      if (prop.regsPerMultiprocessor > 0) {
        // gfx950's file holds, per lane, as many accumulation registers as
        // architectural ones; runtimes differ in whether they count both
        // (ROCm 7.2: 131072 per CU) or the architectural half (7.0: 65536)
        int64_t regs = prop.regsPerMultiprocessor;
        if (regs == 4 * 64 * 256) regs *= 2;
        d.facts.vgpr_bytes_per_cu = regs * 4;
      }
      if (prop.l2CacheSize > 0) d.facts.l2_bytes_per_xcd = (int64_t)prop.l2CacheSize;
      if (prop.clockRate > 0) d.facts.clock_ghz = prop.clockRate * 1e-6;
      int xcc = 0;
      if (hipDeviceGetAttribute(&xcc, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess && xcc > 0)
        d.facts.num_xcds = xcc;
    } else {
      d.status = COSMA_ERR_HIP;
    }
    d.queried = true;
  }
  if (status) *status = d.status;
  return d.facts;
}

bool workspace_for_current(void** ptr, size_t* bytes) {
  const int dev = current_device();
  if (dev < 0) return false;
  std::lock_guard<std::mutex> lock(g_mutex);
  *ptr = g_dev[dev].workspace;
  *bytes = g_dev[dev].workspace_bytes;
  return true;
}

int plan_cached(int64_t m, int64_t n, int64_t k, int dtype, cosma_plan_info* out,
                int64_t a_pitch_bytes) {
  const int dev = current_device();
  int st = COSMA_OK;
  const cosma_device_facts f = device_facts(&st);
  if (a_pitch_bytes <= 0) a_pitch_bytes = k * (int64_t)word_bytes(dtype);
  const auto key = std::make_tuple(dev, m, n, k, dtype, conflicting_pitch(a_pitch_bytes) ? 1 : 0);
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      *out = it->second;
      return COSMA_OK;
    }
  }
  const int rc = make_plan(m, n, k, dtype, f, env_delta(), -1, -1, out, a_pitch_bytes);
  if (rc != COSMA_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_plans.size() > 4096) g_plans.clear();
  g_plans[key] = *out;
  return COSMA_OK;
}

int map_hip(hipError_t e) { return e == hipSuccess ? COSMA_OK : COSMA_ERR_HIP; }

namespace {

bool aligned_to(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

// Argument rules of the header; nothing is launched when this fails.
int check_args(int64_t m, int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, const void* C, int64_t ldc, int dtype) {
  if (dtype < 0 || dtype >= NUM_DTYPES) return COSMA_ERR_INVALID_ARG;
  if (m < 0 || n < 0 || k < 0) return COSMA_ERR_INVALID_ARG;
  if (lda < (k > 1 ? k : 1) || ldb < (n > 1 ? n : 1) || ldc < (n > 1 ? n : 1))
    return COSMA_ERR_INVALID_ARG;
  const size_t el = (size_t)word_bytes(dtype);
  if (m == 0 || n == 0) return COSMA_OK;
  if (!C || !aligned_to(C, el)) return COSMA_ERR_INVALID_ARG;
  // int64 extents must not overflow
  const double lim = 9.0e18;
  if ((double)m * (double)ldc > lim) return COSMA_ERR_INVALID_ARG;
  if (k > 0 && alpha != 0.0) {
    if (!A || !B || !aligned_to(A, el) || !aligned_to(B, el)) return COSMA_ERR_INVALID_ARG;
    if ((double)m * (double)lda > lim || (double)k * (double)ldb > lim) return COSMA_ERR_INVALID_ARG;
  }
  (void)beta;
  return COSMA_OK;
}

namespace {

// BF16x3: split pass into the workspace planes, GEMM, split-K reduction.
int run_bf16x3(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* ws,
               hipStream_t stream) {
  const int64_t m = plan.m, n = plan.n, k = plan.k;
  X3Args g;
  std::memset(&g, 0, sizeof(g));
  g.kp = ceil_div(k, 32) * 32;
  g.rows_p = ceil_div(m, 256) * 256;
  g.cols_p = ceil_div(n, 256) * 256;
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  char* w = static_cast<char*>(ws);
  const size_t part = plan.p_k > 1 ? up((size_t)plan.p_k * m * n * sizeof(float)) : 0;
  unsigned short* base = reinterpret_cast<unsigned short*>(w + part);
  g.a_hi = base;
  g.a_lo = base + (size_t)g.rows_p * g.kp;
  g.b_hi = base + (size_t)2 * g.rows_p * g.kp;
  g.b_lo = base + (size_t)2 * g.rows_p * g.kp + (size_t)g.cols_p * g.kp;
  g.C = C;
  g.P = w;
  g.ldc = ldc;
  g.m = m;
  g.n = n;
  g.k_split = plan.k_split;
  g.tiles_m = plan.p_m;
  g.tiles_n = plan.p_n;
  g.splits = plan.p_k;
  g.ldp = n;
  g.split_stride = m * n;
  g.alpha = alpha;
  g.beta = beta;
  g.group_m = plan.group_m > 0 ? plan.group_m : 1;
  int st = COSMA_OK;
  g.num_xcds = device_facts(&st).num_xcds;
  hipError_t e = launch_bf16x3_split(static_cast<const float*>(A), m, k, lda,
                                     static_cast<const float*>(B), n, ldb, g, stream);
  if (e != hipSuccess) return COSMA_ERR_HIP;
  e = launch_gemm_bf16x3(plan.tile_id, g, stream);
  if (e != hipSuccess) return COSMA_ERR_HIP;
  if (plan.p_k > 1) {
    e = launch_splitk_reduce_f32((const float*)w, m * n, n, plan.p_k, (float*)C, ldc, m, n,
                                 (float)alpha, (float)beta, stream);
    if (e != hipSuccess) return COSMA_ERR_HIP;
  }
  return COSMA_OK;
}

}  // namespace

// Run one product under `plan` (validated by the caller) with the
// registered workspace.
int run_plan(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda, const void* B,
             int64_t ldb, double beta, void* C, int64_t ldc, hipStream_t stream) {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  if (!workspace_for_current(&ws, &ws_bytes)) ws = nullptr, ws_bytes = 0;
  return run_plan_ws(plan, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes, stream);
}

// Run one product under `plan` with the device buffer `ws` of `ws_bytes`
// as its workspace.
int run_plan_ws(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
                const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* ws,
                size_t ws_bytes, hipStream_t stream) {
  const int64_t m = plan.m, n = plan.n, k = plan.k;
  const int dtype = plan.dtype;
  if (m == 0 || n == 0) return COSMA_OK;
  const bool fp32 = dtype == F32 || dtype == F32_BF16X3;
  if (k == 0 || alpha == 0.0) {
    if (fp32) return map_hip(launch_scale_f32((float*)C, ldc, m, n, (float)beta, stream));
    return map_hip(launch_scale_f64((double*)C, ldc, m, n, beta, stream));
  }
  // The requirement is recomputed from the plan's shape, never taken from
  // its (caller-writable) workspace_bytes field.
  const size_t need = workspace_bytes(plan);
  if (need > 0 && (!ws || ws_bytes < need)) return COSMA_ERR_WORKSPACE;
  if (dtype == F64_OZAKI_I8) return run_ozaki(plan, alpha, A, lda, B, ldb, beta, C, ldc, ws, stream);
  if (dtype == F64_OZAKI2_I8)
    return run_ozaki2(plan, alpha, A, lda, B, ldb, beta, C, ldc, ws, stream);
  if (dtype == F64_OZAKI_BF16)
    return run_ozaki_bf16(plan, alpha, A, lda, B, ldb, beta, C, ldc, ws, stream);
  if (dtype == F32_BF16X3) return run_bf16x3(plan, alpha, A, lda, B, ldb, beta, C, ldc, ws, stream);

  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.m = m;
  g.n = n;
  g.k = k;
  g.k_split = plan.k_split;
  g.tiles_m = plan.p_m;
  g.tiles_n = plan.p_n;
  g.splits = plan.p_k;
  g.ldp = n;
  g.split_stride = m * n;
  g.alpha = alpha;
  g.beta = beta;
  g.group_m = plan.group_m > 0 ? plan.group_m : 1;
  int st = COSMA_OK;
  g.num_xcds = device_facts(&st).num_xcds;
  const size_t el = (size_t)word_bytes(dtype);
  // 16-byte loads need a 16-byte aligned base and a row pitch of 16 bytes.
  g.vec_a = ((uintptr_t)A % 16 == 0 && ((size_t)lda * el) % 16 == 0) ? 1 : 0;
  g.vec_b = ((uintptr_t)B % 16 == 0 && ((size_t)ldb * el) % 16 == 0) ? 1 : 0;
  if (plan.p_k > 1) g.P = ws;

  hipError_t e;
  switch (dtype) {
    case F64: e = launch_gemm_f64(plan.tile_id, g, stream); break;
    case F32: e = launch_gemm_f32(plan.tile_id, g, stream); break;
    default: return COSMA_ERR_INVALID_ARG;
  }
  if (e != hipSuccess) return COSMA_ERR_HIP;
  if (plan.p_k > 1) {
    if (fp32)
      e = launch_splitk_reduce_f32((const float*)ws, m * n, n, plan.p_k, (float*)C, ldc, m, n,
                                   (float)alpha, (float)beta, stream);
    else
      e = launch_splitk_reduce_f64((const double*)ws, m * n, n, plan.p_k, (double*)C, ldc, m, n,
                                   alpha, beta, stream);
    if (e != hipSuccess) return COSMA_ERR_HIP;
  }
  return COSMA_OK;
}

int check_plan(const cosma_plan_info* p) {
  if (!p) return COSMA_ERR_INVALID_ARG;
  int cnt = 0;
  const TileDesc* menu = tile_menu(p->dtype, &cnt);
  if (!menu || p->tile_id < 0 || p->tile_id >= cnt) return COSMA_ERR_INVALID_ARG;
  const TileDesc& T = menu[p->tile_id];
  if (p->m < 0 || p->n < 0 || p->k < 0) return COSMA_ERR_INVALID_ARG;
  if (p->m == 0 || p->n == 0 || p->k == 0) return COSMA_OK;
  if (p->tile_m != T.tm || p->tile_n != T.tn || p->tile_k != T.tk) return COSMA_ERR_INVALID_ARG;
  if (p->p_m != ceil_div(p->m, T.tm) || p->p_n != ceil_div(p->n, T.tn)) return COSMA_ERR_INVALID_ARG;
  if (p->p_k < 1 || p->k_split < T.tk || p->k_split % T.tk) return COSMA_ERR_INVALID_ARG;
  if (ceil_div(p->k, p->k_split) != p->p_k) return COSMA_ERR_INVALID_ARG;
  if (p->group_m < 1) return COSMA_ERR_INVALID_ARG;
  if ((p->dtype == F64_OZAKI_I8 || p->dtype == F64_OZAKI_BF16) && (p->slices < 1 || p->slices > 8))
    return COSMA_ERR_INVALID_ARG;
  if (p->dtype == F64_OZAKI2_I8 &&
      (p->slices < CRT_MIN_MODULI || p->slices > CRT_MAX_MODULI || p->k_split > OZAKI2_MAX_K_ITEM))
    return COSMA_ERR_INVALID_ARG;
  return COSMA_OK;
}

namespace {

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// CBLAS arguments brought to the row-major, no-transpose form of the
// kernels: a column-major product C = op(A) op(B) is the row-major product
// C^T = op(B)^T op(A)^T on the same memory, so layout swaps the operands,
// their flags and m, n.  On return `ta` / `tb` say whether A / B (after the
// swap) are stored transposed.  Leading dimensions are checked here.
struct ExArgs {
  int64_t m, n, k;
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  bool ta, tb;
};

int normalise_ex(int layout, int transa, int transb, int64_t m, int64_t n, int64_t k,
                 const void* A, int64_t lda, const void* B, int64_t ldb, int64_t ldc,
                 ExArgs* out) {
  if ((layout != COSMA_ROW_MAJOR && layout != COSMA_COL_MAJOR) ||
      (transa != COSMA_NO_TRANS && transa != COSMA_TRANS) ||
      (transb != COSMA_NO_TRANS && transb != COSMA_TRANS))
    return COSMA_ERR_INVALID_ARG;
  if (m < 0 || n < 0 || k < 0) return COSMA_ERR_INVALID_ARG;
  ExArgs e;
  if (layout == COSMA_ROW_MAJOR) {
    e = ExArgs{m, n, k, A, lda, B, ldb, transa == COSMA_TRANS, transb == COSMA_TRANS};
  } else {
    e = ExArgs{n, m, k, B, ldb, A, lda, transb == COSMA_TRANS, transa == COSMA_TRANS};
  }
  // row-major: op(A) is m x k (stored k x m when transposed), op(B) k x n
  const int64_t need_a = e.ta ? e.m : e.k, need_b = e.tb ? e.k : e.n;
  if (e.lda < (need_a > 1 ? need_a : 1) || e.ldb < (need_b > 1 ? need_b : 1) ||
      ldc < (e.n > 1 ? e.n : 1))
    return COSMA_ERR_INVALID_ARG;
  *out = e;
  return COSMA_OK;
}

// Workspace of the product's plan followed by the transposed copies.
size_t ex_workspace(const cosma_plan_info& plan, const ExArgs& e, int dtype) {
  const size_t w = (size_t)word_bytes(dtype);
  size_t ws = up256(workspace_bytes(plan));
  if (e.ta) ws += up256((size_t)e.m * (size_t)e.k * w);
  if (e.tb) ws += up256((size_t)e.k * (size_t)e.n * w);
  return ws;
}

bool products_needed(const ExArgs& e, double alpha) {
  return e.m > 0 && e.n > 0 && e.k > 0 && alpha != 0.0;
}

// ScaLAPACK array descriptor of a dense matrix: DTYPE_, CTXT_, M_, N_, MB_,
// NB_, RSRC_, CSRC_, LLD_.
enum { DESC_DTYPE = 0, DESC_M = 2, DESC_N = 3, DESC_MB = 4, DESC_NB = 5, DESC_RSRC = 6,
       DESC_CSRC = 7, DESC_LLD = 8 };

// The rows x cols block of a descriptor-described matrix that starts at the
// 1-based global position (i, j).  On a 1 x 1 process grid every block of the
// block-cyclic distribution is local and the local array is the whole matrix,
// column-major with leading dimension LLD_, whatever MB_ and NB_ are; *sub is
// the block's first element (null if X is null).
int sub_block(const void* X, int64_t i, int64_t j, const int32_t* desc, int64_t rows, int64_t cols,
              size_t el, const void** sub, int64_t* ld) {
  if (!desc || desc[DESC_DTYPE] != 1) return COSMA_ERR_INVALID_ARG;
  const int64_t M = desc[DESC_M], N = desc[DESC_N], lld = desc[DESC_LLD];
  if (M < 0 || N < 0 || desc[DESC_MB] < 1 || desc[DESC_NB] < 1) return COSMA_ERR_INVALID_ARG;
  if (desc[DESC_RSRC] != 0 || desc[DESC_CSRC] != 0) return COSMA_ERR_INVALID_ARG;
  if (lld < (M > 1 ? M : 1) || i < 1 || j < 1) return COSMA_ERR_INVALID_ARG;
  if (rows > 0 && cols > 0 && (i - 1 + rows > M || j - 1 + cols > N)) return COSMA_ERR_INVALID_ARG;
  *ld = lld;
  *sub = X ? static_cast<const char*>(X) + ((j - 1) * lld + (i - 1)) * (int64_t)el : nullptr;
  return COSMA_OK;
}

}  // namespace

}  // namespace cosma

using namespace cosma;

extern "C" {

int cosma_gemm(int64_t m, int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, void* C, int64_t ldc, int dtype,
               void* stream) {
  int rc = check_args(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
  if (rc != COSMA_OK) return rc;
  if (m == 0 || n == 0) return COSMA_OK;
  int st = COSMA_OK;
  device_facts(&st);
  if (st != COSMA_OK) return st;
  cosma_plan_info plan;
  rc = plan_cached(m, n, k, dtype, &plan, lda * (int64_t)word_bytes(dtype));
  if (rc != COSMA_OK) return rc;
  return run_plan(plan, alpha, A, lda, B, ldb, beta, C, ldc, (hipStream_t)stream);
}

int cosma_gemm_planned(const cosma_plan_info* plan, double alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                       void* stream) {
  int rc = check_plan(plan);
  if (rc != COSMA_OK) return rc;
  rc = check_args(plan->m, plan->n, plan->k, alpha, A, lda, B, ldb, beta, C, ldc, plan->dtype);
  if (rc != COSMA_OK) return rc;
  if (plan->m == 0 || plan->n == 0) return COSMA_OK;
  int st = COSMA_OK;
  device_facts(&st);
  if (st != COSMA_OK) return st;
  return run_plan(*plan, alpha, A, lda, B, ldb, beta, C, ldc, (hipStream_t)stream);
}

int cosma_gemm_ex(int layout, int transa, int transb, int64_t m, int64_t n, int64_t k,
                  double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                  double beta, void* C, int64_t ldc, int dtype, void* stream) {
  if (dtype < 0 || dtype >= NUM_DTYPES) return COSMA_ERR_INVALID_ARG;
  ExArgs e;
  int rc = normalise_ex(layout, transa, transb, m, n, k, A, lda, B, ldb, ldc, &e);
  if (rc != COSMA_OK) return rc;
  if (!e.ta && !e.tb)
    return cosma_gemm(e.m, e.n, e.k, alpha, e.A, e.lda, e.B, e.ldb, beta, C, ldc, dtype, stream);
  // operands as the row-major kernels see them: op(A) m x k, op(B) k x n
  const int64_t lda_k = e.ta ? (e.k > 1 ? e.k : 1) : e.lda;
  const int64_t ldb_k = e.tb ? (e.n > 1 ? e.n : 1) : e.ldb;
  const size_t el = (size_t)word_bytes(dtype);
  if (e.m == 0 || e.n == 0) return COSMA_OK;
  if (!C || (uintptr_t)C % el) return COSMA_ERR_INVALID_ARG;
  if (products_needed(e, alpha) &&
      (!e.A || !e.B || (uintptr_t)e.A % el || (uintptr_t)e.B % el))
    return COSMA_ERR_INVALID_ARG;
  if (!products_needed(e, alpha))  // C = beta C, A and B not read
    return cosma_gemm(e.m, e.n, e.k, alpha, e.A, lda_k, e.B, ldb_k, beta, C, ldc, dtype, stream);
  int st = COSMA_OK;
  device_facts(&st);
  if (st != COSMA_OK) return st;
  cosma_plan_info plan;
  rc = plan_cached(e.m, e.n, e.k, dtype, &plan,
                   e.ta ? e.k * (int64_t)el : e.lda * (int64_t)el);
  if (rc != COSMA_OK) return rc;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  if (!workspace_for_current(&ws, &ws_bytes) || !ws || ws_bytes < ex_workspace(plan, e, dtype))
    return COSMA_ERR_WORKSPACE;
  char* tail = static_cast<char*>(ws) + up256(workspace_bytes(plan));
  const void* Ak = e.A;
  const void* Bk = e.B;
  hipStream_t s = (hipStream_t)stream;
  hipError_t err = hipSuccess;
  if (e.ta) {  // A is stored k x m
    if (el == 8)
      err = launch_transpose_f64((const double*)e.A, e.k, e.m, e.lda, (double*)tail, s);
    else
      err = launch_transpose_f32((const float*)e.A, e.k, e.m, e.lda, (float*)tail, s);
    Ak = tail;
    tail += up256((size_t)e.m * (size_t)e.k * el);
  }
  if (err == hipSuccess && e.tb) {  // B is stored n x k
    if (el == 8)
      err = launch_transpose_f64((const double*)e.B, e.n, e.k, e.ldb, (double*)tail, s);
    else
      err = launch_transpose_f32((const float*)e.B, e.n, e.k, e.ldb, (float*)tail, s);
    Bk = tail;
  }
  if (err != hipSuccess) return COSMA_ERR_HIP;
  return run_plan(plan, alpha, Ak, lda_k, Bk, ldb_k, beta, C, ldc, s);
}

int cosma_workspace_size_ex(int layout, int transa, int transb, int64_t m, int64_t n, int64_t k,
                            int dtype, size_t* bytes) {
  if (!bytes || dtype < 0 || dtype >= NUM_DTYPES) return COSMA_ERR_INVALID_ARG;
  ExArgs e;
  // leading dimensions do not matter for the size: pass the smallest legal
  const int64_t lda_min = layout == COSMA_ROW_MAJOR ? (transa == COSMA_TRANS ? m : k)
                                                    : (transa == COSMA_TRANS ? k : m);
  const int64_t ldb_min = layout == COSMA_ROW_MAJOR ? (transb == COSMA_TRANS ? k : n)
                                                    : (transb == COSMA_TRANS ? n : k);
  const int64_t ldc_min = layout == COSMA_ROW_MAJOR ? n : m;
  const int rc = normalise_ex(layout, transa, transb, m, n, k, nullptr,
                              lda_min > 1 ? lda_min : 1, nullptr, ldb_min > 1 ? ldb_min : 1,
                              ldc_min > 1 ? ldc_min : 1, &e);
  if (rc != COSMA_OK) return rc;
  cosma_plan_info plan;
  const int prc = cosma_plan_query(e.m, e.n, e.k, dtype, &plan);
  if (prc != COSMA_OK) return prc;
  *bytes = (e.ta || e.tb) && e.m > 0 && e.n > 0 && e.k > 0 ? ex_workspace(plan, e, dtype)
                                                            : plan.workspace_bytes;
  return COSMA_OK;
}

int cosma_pgemm(int transa, int transb, int64_t m, int64_t n, int64_t k, double alpha,
                const void* A, int64_t ia, int64_t ja, const int32_t* desca, const void* B,
                int64_t ib, int64_t jb, const int32_t* descb, double beta, void* C, int64_t ic,
                int64_t jc, const int32_t* descc, int dtype, void* stream) {
  if (dtype < 0 || dtype >= NUM_DTYPES || m < 0 || n < 0 || k < 0) return COSMA_ERR_INVALID_ARG;
  if ((transa != COSMA_NO_TRANS && transa != COSMA_TRANS) ||
      (transb != COSMA_NO_TRANS && transb != COSMA_TRANS))
    return COSMA_ERR_INVALID_ARG;
  const size_t el = (size_t)word_bytes(dtype);
  const bool ta = transa == COSMA_TRANS, tb = transb == COSMA_TRANS;
  const void *a = nullptr, *b = nullptr, *c = nullptr;
  int64_t lda = 0, ldb = 0, ldc = 0;
  int rc = sub_block(A, ia, ja, desca, ta ? k : m, ta ? m : k, el, &a, &lda);
  if (rc == COSMA_OK) rc = sub_block(B, ib, jb, descb, tb ? n : k, tb ? k : n, el, &b, &ldb);
  if (rc == COSMA_OK) rc = sub_block(C, ic, jc, descc, m, n, el, &c, &ldc);
  if (rc != COSMA_OK) return rc;
  return cosma_gemm_ex(COSMA_COL_MAJOR, transa, transb, m, n, k, alpha, a, lda, b, ldb, beta,
                       const_cast<void*>(c), ldc, dtype, stream);
}

int cosma_plan_query(int64_t m, int64_t n, int64_t k, int dtype, cosma_plan_info* out) {
  if (!out) return COSMA_ERR_INVALID_ARG;
  if (dtype < 0 || dtype >= NUM_DTYPES || m < 0 || n < 0 || k < 0) return COSMA_ERR_INVALID_ARG;
  return plan_cached(m, n, k, dtype, out);
}

int cosma_plan_query_facts(int64_t m, int64_t n, int64_t k, int dtype,
                           const cosma_device_facts* facts, double delta, cosma_plan_info* out) {
  if (!out) return COSMA_ERR_INVALID_ARG;
  cosma_device_facts f;
  if (facts) {
    f = *facts;
  } else {
    int st;
    f = device_facts(&st);
  }
  return make_plan(m, n, k, dtype, f, delta, -1, -1, out);
}

int cosma_plan_make(int64_t m, int64_t n, int64_t k, int dtype, int tile_id, int p_k,
                    cosma_plan_info* out) {
  if (!out || tile_id < 0 || p_k < 1) return COSMA_ERR_INVALID_ARG;
  int st;
  const cosma_device_facts f = device_facts(&st);
  const int rc = make_plan(m, n, k, dtype, f, env_delta(), tile_id, p_k, out);
  if (rc != COSMA_OK) return rc;
  if (m > 0 && n > 0 && k > 0 && out->p_k != p_k) return COSMA_ERR_INVALID_ARG;  // k too short
  return COSMA_OK;
}

int cosma_plan_set_slices(cosma_plan_info* plan, int slices) {
  if (!plan) return COSMA_ERR_INVALID_ARG;
  if (plan->dtype == F64_OZAKI_I8 || plan->dtype == F64_OZAKI_BF16) {
    if (slices < 1 || slices > 8) return COSMA_ERR_INVALID_ARG;
  } else if (plan->dtype == F64_OZAKI2_I8) {
    if (slices < CRT_MIN_MODULI || slices > CRT_MAX_MODULI) return COSMA_ERR_INVALID_ARG;
    CrtParams cp;  // too few moduli leave no operand bits at this k
    if (plan->k > 0 && !crt_params(plan->k, slices, &cp)) return COSMA_ERR_INVALID_ARG;
    // one GEMM per modulus and split and tile
    if (plan->p_m > 0 && plan->p_n > 0)
      plan->items = (int64_t)plan->p_m * plan->p_n * plan->p_k * slices;
  } else {
    return COSMA_ERR_INVALID_ARG;
  }
  plan->slices = slices;
  plan->workspace_bytes = workspace_bytes(*plan);
  set_error_contract(plan);
  return COSMA_OK;
}

int cosma_set_ozaki_spread(double spread) {
  if (!set_ozaki_target_spread(spread)) return COSMA_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mutex);
  g_plans.clear();
  return COSMA_OK;
}

int cosma_get_ozaki_spread(double* spread) {
  if (!spread) return COSMA_ERR_INVALID_ARG;
  *spread = ozaki_target_spread();
  return COSMA_OK;
}

int cosma_ozaki2_params(int64_t k, int nmod, int32_t* beta, int32_t* moduli) {
  if (!beta || !moduli) return COSMA_ERR_INVALID_ARG;
  CrtParams cp;
  if (!crt_params(k, nmod, &cp)) return COSMA_ERR_INVALID_ARG;
  *beta = cp.beta;
  for (int l = 0; l < nmod; ++l) moduli[l] = cp.p[l];
  return COSMA_OK;
}

int cosma_tile_count(int dtype) {
  int c = 0;
  tile_menu(dtype, &c);
  return c;
}

int cosma_tile_shape(int dtype, int id, int32_t* tm, int32_t* tn, int32_t* tk) {
  int c = 0;
  const TileDesc* menu = tile_menu(dtype, &c);
  if (!menu || id < 0 || id >= c || !tm || !tn || !tk) return COSMA_ERR_INVALID_ARG;
  *tm = menu[id].tm;
  *tn = menu[id].tn;
  *tk = menu[id].tk;
  return COSMA_OK;
}

int cosma_device_query(cosma_device_facts* out) {
  if (!out) return COSMA_ERR_INVALID_ARG;
  int st = COSMA_OK;
  *out = device_facts(&st);
  return st;
}

double cosma_thm1_bound(double m, double n, double k, double S) {
  if (!(S > 0)) return NAN;
  return thm1_bound(m, n, k, S);
}

int cosma_seq_schedule(int64_t S, int64_t* a, int64_t* b) {
  if (S < 3 || !a || !b) return COSMA_ERR_INVALID_ARG;
  seq_schedule(S, a, b);
  return COSMA_OK;
}

int cosma_par_schedule(double m, double n, double k, double p, double S, double* a, double* b) {
  if (!(m > 0 && n > 0 && k > 0 && p > 0 && S > 0) || !a || !b) return COSMA_ERR_INVALID_ARG;
  par_schedule(m, n, k, p, S, a, b);
  return COSMA_OK;
}

int cosma_fit_ranks(int64_t m, int64_t n, int64_t k, int64_t p, double delta, int64_t grid[3],
                    int64_t* used) {
  if (!grid || !used) return COSMA_ERR_INVALID_ARG;
  return fit_ranks(m, n, k, p, delta, grid, used) ? COSMA_OK : COSMA_ERR_INVALID_ARG;
}

double cosma_io_count(int64_t m, int64_t n, int64_t k, int64_t tm, int64_t tn, int64_t kc,
                      int64_t pk, int beta_nonzero) {
  return io_count(m, n, k, tm, tn, kc, pk, beta_nonzero != 0);
}

int cosma_workspace_size(int64_t m, int64_t n, int64_t k, int dtype, size_t* bytes) {
  if (!bytes) return COSMA_ERR_INVALID_ARG;
  cosma_plan_info p;
  const int rc = cosma_plan_query(m, n, k, dtype, &p);
  if (rc != COSMA_OK) return rc;
  *bytes = p.workspace_bytes;
  return COSMA_OK;
}

int cosma_set_workspace(void* ptr, size_t bytes, void* stream) {
  (void)stream;
  if ((ptr == nullptr) != (bytes == 0)) return COSMA_ERR_INVALID_ARG;
  if (ptr && ((uintptr_t)ptr % 256) != 0) return COSMA_ERR_INVALID_ARG;
  const int dev = current_device();
  if (dev < 0) return COSMA_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mutex);
  g_dev[dev].workspace = ptr;
  g_dev[dev].workspace_bytes = bytes;
  return COSMA_OK;
}

const char* cosma_status_string(int status) {
  switch (status) {
    case COSMA_OK: return "COSMA_OK";
    case COSMA_ERR_INVALID_ARG: return "COSMA_ERR_INVALID_ARG: invalid argument";
    case COSMA_ERR_HIP: return "COSMA_ERR_HIP: a HIP runtime call failed";
    case COSMA_ERR_WORKSPACE: return "COSMA_ERR_WORKSPACE: registered workspace too small";
    case COSMA_ERR_UNSUPPORTED: return "COSMA_ERR_UNSUPPORTED: no gfx950 device or unsupported case";
    case COSMA_ERR_NO_MEMORY: return "COSMA_ERR_NO_MEMORY: host allocation failed";
    default: return "unknown cosma status";
  }
}

const char* cosma_version(void) { return "cosma_mi355 0.1.0 (gfx950)"; }

}  // extern "C"
