"""Python binding of the cosma_mi355 C ABI (``include/cosma_mi355.h``).

Argument marshalling only: every step of a product runs in the HIP library
``libcosma_mi355.so``.  The functions below carry the C names; device
pointers may be given as integers or as torch tensors (their ``data_ptr()``),
streams as integers, torch streams, or ``None`` (torch's current stream).
PyTorch serves only as the source of device memory and streams.

There is no fallback: if the library is missing every call raises.
"""
from __future__ import annotations

import array
import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcosma_mi355.so")

COSMA_F64 = 0
COSMA_F32 = 1
COSMA_F32_BF16X3 = 2
COSMA_F64_OZAKI_I8 = 3
COSMA_F64_OZAKI2_I8 = 4
COSMA_F64_OZAKI_BF16 = 5
DTYPES = {"f64": COSMA_F64, "f32": COSMA_F32, "bf16x3": COSMA_F32_BF16X3, "ozaki": COSMA_F64_OZAKI_I8,
          "ozaki2": COSMA_F64_OZAKI2_I8, "ozaki_bf16": COSMA_F64_OZAKI_BF16}

COSMA_ROW_MAJOR = 0
COSMA_COL_MAJOR = 1
COSMA_NO_TRANS = 0
COSMA_TRANS = 1

COSMA_OK = 0
COSMA_ERR_INVALID_ARG = -1
COSMA_ERR_HIP = -2
COSMA_ERR_WORKSPACE = -3
COSMA_ERR_UNSUPPORTED = -4
COSMA_ERR_NO_MEMORY = -5

EXPORTED = [
    "cosma_gemm", "cosma_gemm_planned", "cosma_gemm_noalloc", "cosma_gemm_ex", "cosma_workspace_size_ex", "cosma_pgemm",
    "cosma_gemm_batched", "cosma_batch_create",
    "cosma_batch_run", "cosma_batch_destroy", "cosma_batch_info", "cosma_batch_tuning", "cosma_batch_tiles",
    "cosma_batch_splits", "cosma_workspace_size_batched", "cosma_plan_query", "cosma_plan_query_facts",
    "cosma_plan_make", "cosma_plan_set_slices", "cosma_set_ozaki_spread", "cosma_get_ozaki_spread", "cosma_ozaki2_params", "cosma_tile_count", "cosma_tile_shape", "cosma_device_query",
    "cosma_thm1_bound", "cosma_seq_schedule", "cosma_par_schedule", "cosma_fit_ranks",
    "cosma_io_count", "cosma_workspace_size", "cosma_set_workspace", "cosma_status_string",
    "cosma_version",
]


class CosmaError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {cosma_status_string(status)} ({status})" if what else
                         f"{cosma_status_string(status)} ({status})")


class cosma_device_facts(ctypes.Structure):
    _fields_ = [("num_cus", ctypes.c_int32), ("num_xcds", ctypes.c_int32),
                ("lds_bytes_per_cu", ctypes.c_int64), ("vgpr_bytes_per_cu", ctypes.c_int64),
                ("l2_bytes_per_xcd", ctypes.c_int64), ("clock_ghz", ctypes.c_double),
                ("hbm_gbps", ctypes.c_double)]


class cosma_plan_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("tile_id", ctypes.c_int32),
                ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32), ("tile_k", ctypes.c_int32),
                ("p_m", ctypes.c_int32), ("p_n", ctypes.c_int32), ("p_k", ctypes.c_int32),
                ("group_m", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("regime", ctypes.c_int32), ("slices", ctypes.c_int32),
                ("k_split", ctypes.c_int64), ("items", ctypes.c_int64), ("waves", ctypes.c_int64),
                ("S_words", ctypes.c_double), ("p1", ctypes.c_double),
                ("a_seq", ctypes.c_int64), ("b_seq", ctypes.c_int64),
                ("a_par", ctypes.c_double), ("b_par", ctypes.c_double),
                ("q_cu_words", ctypes.c_double), ("q_ea_bytes", ctypes.c_double),
                ("thm1_words", ctypes.c_double), ("thm2_words", ctypes.c_double),
                ("predicted_ms", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t),
                ("err_scaled", ctypes.c_double), ("err_rounding", ctypes.c_double),
                ("spread_limit", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -c 'import __graft_entry__ as g; g.build()'`")
            L = ctypes.CDLL(LIB_PATH)
            i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
            pi64, pdbl, ppv = ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(vp)
            pi32 = ctypes.POINTER(ctypes.c_int32)
            P = ctypes.POINTER(cosma_plan_info)
            sig = {
                "cosma_gemm": (i32, [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, i32, vp]),
                "cosma_gemm_planned": (i32, [P, dbl, vp, i64, vp, i64, dbl, vp, i64, vp]),
                "cosma_gemm_noalloc": (i32, [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64,
                                             i32, vp]),
                "cosma_gemm_ex": (i32, [i32, i32, i32, i64, i64, i64, dbl, vp, i64, vp, i64, dbl,
                                        vp, i64, i32, vp]),
                "cosma_workspace_size_ex": (i32, [i32, i32, i32, i64, i64, i64, i32,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
                "cosma_pgemm": (i32, [i32, i32, i64, i64, i64, dbl, vp, i64, i64, pi32, vp, i64,
                                      i64, pi32, dbl, vp, i64, i64, pi32, i32, vp]),
                "cosma_gemm_batched": (i32, [i64, pi64, pi64, pi64, pdbl, ppv, pi64, ppv, pi64,
                                             pdbl, ppv, pi64, i32, vp]),
                "cosma_batch_create": (i32, [i64, pi64, pi64, pi64, pdbl, ppv, pi64, ppv, pi64,
                                             pdbl, ppv, pi64, i32, vp, ctypes.POINTER(vp)]),
                "cosma_batch_run": (i32, [vp, vp]),
                "cosma_batch_destroy": (i32, [vp]),
                "cosma_batch_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), pi64,
                                           pdbl, i32]),
                "cosma_batch_tuning": (i32, [vp, ctypes.POINTER(i32), pdbl, pdbl]),
                "cosma_batch_tiles": (i32, [vp, i64, ctypes.POINTER(ctypes.c_int32)]),
                "cosma_batch_splits": (i32, [vp, i64, ctypes.POINTER(ctypes.c_int32)]),
                "cosma_workspace_size_batched": (i32, [i64, pi64, pi64, pi64, pdbl, i32,
                                                       ctypes.POINTER(ctypes.c_size_t)]),
                "cosma_plan_query": (i32, [i64, i64, i64, i32, P]),
                "cosma_plan_query_facts": (i32, [i64, i64, i64, i32,
                                                 ctypes.POINTER(cosma_device_facts), dbl, P]),
                "cosma_plan_make": (i32, [i64, i64, i64, i32, i32, i32, P]),
                "cosma_plan_set_slices": (i32, [P, i32]),
                "cosma_set_ozaki_spread": (i32, [dbl]),
                "cosma_get_ozaki_spread": (i32, [pdbl]),
                "cosma_ozaki2_params": (i32, [i64, i32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
                "cosma_tile_count": (i32, [i32]),
                "cosma_tile_shape": (i32, [i32, i32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]),
                "cosma_device_query": (i32, [ctypes.POINTER(cosma_device_facts)]),
                "cosma_thm1_bound": (dbl, [dbl, dbl, dbl, dbl]),
                "cosma_seq_schedule": (i32, [i64, pi64, pi64]),
                "cosma_par_schedule": (i32, [dbl, dbl, dbl, dbl, dbl, pdbl, pdbl]),
                "cosma_fit_ranks": (i32, [i64, i64, i64, i64, dbl, pi64, pi64]),
                "cosma_io_count": (dbl, [i64, i64, i64, i64, i64, i64, i64, i32]),
                "cosma_workspace_size": (i32, [i64, i64, i64, i32, ctypes.POINTER(ctypes.c_size_t)]),
                "cosma_set_workspace": (i32, [vp, ctypes.c_size_t, vp]),
                "cosma_status_string": (ctypes.c_char_p, [i32]),
                "cosma_version": (ctypes.c_char_p, []),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


# ------------------------------------------------------------ marshalling
def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    raise TypeError(f"cannot take a device pointer of {type(x)}")


def _stream(s) -> int | None:
    if s is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return s
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    raise TypeError(f"cannot take a stream handle of {type(s)}")


def _dtype(d) -> int:
    return DTYPES[d] if isinstance(d, str) else int(d)


# Arrays for the batched calls are built through the array module (one C
# conversion pass) and handed to ctypes without a copy; the ctypes object
# keeps the array alive.
def _carray(ctype, code, values):
    if not values:
        return (ctype * 0)()
    a = array.array(code, values)
    return (ctype * len(a)).from_buffer(a)


def _i64arr(v):
    v = list(v)
    try:
        return _carray(ctypes.c_int64, "q", v)
    except TypeError:  # values that are not integers: converted one by one
        return _carray(ctypes.c_int64, "q", [int(x) for x in v])


def _dblarr(v):
    v = list(v)
    try:
        return _carray(ctypes.c_double, "d", v)
    except TypeError:
        return _carray(ctypes.c_double, "d", [float(x) for x in v])


def _ptrarr(v):
    v = list(v)
    try:  # all tensors
        return _carray(ctypes.c_void_p, "Q", [x.data_ptr() for x in v])
    except AttributeError:
        return _carray(ctypes.c_void_p, "Q", [_ptr(x) or 0 for x in v])


# ------------------------------------------------------------ C names
def cosma_status_string(status: int) -> str:
    return lib().cosma_status_string(int(status)).decode()


def cosma_version() -> str:
    return lib().cosma_version().decode()


def cosma_gemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, stream=None) -> int:
    return lib().cosma_gemm(m, n, k, float(alpha), _ptr(A), lda, _ptr(B), ldb, float(beta),
                            _ptr(C), ldc, _dtype(dtype), _stream(stream))


NOALLOC_SCRATCH_BYTES = 64 << 20  # COSMA_NOALLOC_SCRATCH_BYTES


def cosma_gemm_noalloc(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, stream=None) -> int:
    return lib().cosma_gemm_noalloc(m, n, k, float(alpha), _ptr(A), lda, _ptr(B), ldb,
                                    float(beta), _ptr(C), ldc, _dtype(dtype), _stream(stream))


def cosma_gemm_planned(plan, alpha, A, lda, B, ldb, beta, C, ldc, stream=None) -> int:
    return lib().cosma_gemm_planned(ctypes.byref(plan), float(alpha), _ptr(A), lda, _ptr(B), ldb,
                                    float(beta), _ptr(C), ldc, _stream(stream))


def cosma_gemm_ex(layout, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype,
                  stream=None) -> int:
    return lib().cosma_gemm_ex(int(layout), int(transa), int(transb), m, n, k, float(alpha),
                               _ptr(A), lda, _ptr(B), ldb, float(beta), _ptr(C), ldc,
                               _dtype(dtype), _stream(stream))


def descinit(m, n, mb, nb, lld):
    """ScaLAPACK array descriptor of an m x n dense matrix on the 1 x 1 grid
    (DTYPE_ 1, context 0, first block on process row / column 0)."""
    return [1, 0, int(m), int(n), int(mb), int(nb), 0, 0, int(lld)]


def _desc(d):
    return None if d is None else (ctypes.c_int32 * len(d))(*[int(x) for x in d])


def cosma_pgemm(transa, transb, m, n, k, alpha, A, ia, ja, desca, B, ib, jb, descb, beta, C, ic,
                jc, descc, dtype, stream=None) -> int:
    return lib().cosma_pgemm(int(transa), int(transb), m, n, k, float(alpha), _ptr(A), ia, ja,
                             _desc(desca), _ptr(B), ib, jb, _desc(descb), float(beta), _ptr(C),
                             ic, jc, _desc(descc), _dtype(dtype), _stream(stream))


def cosma_workspace_size_ex(layout, transa, transb, m, n, k, dtype):
    b = ctypes.c_size_t()
    rc = lib().cosma_workspace_size_ex(int(layout), int(transa), int(transb), m, n, k,
                                       _dtype(dtype), ctypes.byref(b))
    return rc, b.value


def cosma_gemm_batched(count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype,
                       stream=None) -> int:
    return lib().cosma_gemm_batched(count, _i64arr(m), _i64arr(n), _i64arr(k), _dblarr(alpha),
                                    _ptrarr(A), _i64arr(lda), _ptrarr(B), _i64arr(ldb),
                                    _dblarr(beta), _ptrarr(C), _i64arr(ldc), _dtype(dtype),
                                    _stream(stream))


def cosma_batch_create(count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, stream=None):
    """Returns (status, handle)."""
    h = ctypes.c_void_p()
    rc = lib().cosma_batch_create(count, _i64arr(m), _i64arr(n), _i64arr(k), _dblarr(alpha),
                                  _ptrarr(A), _i64arr(lda), _ptrarr(B), _i64arr(ldb),
                                  _dblarr(beta), _ptrarr(C), _i64arr(ldc), _dtype(dtype),
                                  _stream(stream), ctypes.byref(h))
    return rc, h.value


def cosma_batch_run(handle, stream=None) -> int:
    return lib().cosma_batch_run(handle, _stream(stream))


def cosma_batch_destroy(handle) -> int:
    return lib().cosma_batch_destroy(handle)


BATCH_POLICIES = 6
BATCH_POLICY_DEFAULT = 5  # one tile for the whole batch; what the one-shot call and an untuned handle use


def cosma_batch_info(handle):
    """Returns (status, policy, groups, items, [ms per candidate policy])."""
    pol, groups, items = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    ms = (ctypes.c_double * BATCH_POLICIES)()
    rc = lib().cosma_batch_info(handle, ctypes.byref(pol), ctypes.byref(groups),
                                ctypes.byref(items), ms, BATCH_POLICIES)
    return rc, pol.value, groups.value, items.value, list(ms)


def cosma_batch_tuning(handle):
    """Returns (status, refinement trials, fastest policy's ms, kept ms)."""
    trials, seed, tuned = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    rc = lib().cosma_batch_tuning(handle, ctypes.byref(trials), ctypes.byref(seed),
                                  ctypes.byref(tuned))
    return rc, trials.value, seed.value, tuned.value


def cosma_batch_tiles(handle, count):
    """Returns (status, [tile id per input problem])."""
    out = (ctypes.c_int32 * max(1, count))()
    rc = lib().cosma_batch_tiles(handle, count, out)
    return rc, list(out)[:count]


def cosma_batch_splits(handle, count):
    """Returns (status, [split factor per input problem])."""
    out = (ctypes.c_int32 * max(1, count))()
    rc = lib().cosma_batch_splits(handle, count, out)
    return rc, list(out)[:count]


def cosma_workspace_size_batched(count, m, n, k, alpha, dtype):
    """Returns (status, bytes) for cosma_gemm_batched."""
    b = ctypes.c_size_t()
    rc = lib().cosma_workspace_size_batched(count, _i64arr(m), _i64arr(n), _i64arr(k),
                                            _dblarr(alpha), _dtype(dtype), ctypes.byref(b))
    return rc, b.value


def gemm_batched(count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, stream=None) -> int:
    """cosma_gemm_batched with the workspace it needs registered first."""
    rc, ws = cosma_workspace_size_batched(count, m, n, k, alpha, dtype)
    if rc != COSMA_OK:
        return rc
    if ws:
        ensure_workspace(ws)
    return cosma_gemm_batched(count, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, stream)


def cosma_plan_query(m, n, k, dtype):
    """Returns (status, cosma_plan_info)."""
    p = cosma_plan_info()
    rc = lib().cosma_plan_query(m, n, k, _dtype(dtype), ctypes.byref(p))
    return rc, p


def cosma_plan_query_facts(m, n, k, dtype, facts=None, delta=0.03):
    p = cosma_plan_info()
    fp = ctypes.byref(facts) if facts is not None else None
    rc = lib().cosma_plan_query_facts(m, n, k, _dtype(dtype), fp, float(delta), ctypes.byref(p))
    return rc, p


def cosma_plan_make(m, n, k, dtype, tile_id, p_k):
    p = cosma_plan_info()
    rc = lib().cosma_plan_make(m, n, k, _dtype(dtype), tile_id, p_k, ctypes.byref(p))
    return rc, p


def cosma_plan_set_slices(plan, slices) -> int:
    return lib().cosma_plan_set_slices(ctypes.byref(plan), int(slices))


def cosma_set_ozaki_spread(spread) -> int:
    return lib().cosma_set_ozaki_spread(float(spread))


def cosma_get_ozaki_spread():
    """Returns (status, target spread)."""
    v = ctypes.c_double()
    rc = lib().cosma_get_ozaki_spread(ctypes.byref(v))
    return rc, v.value


def cosma_ozaki2_params(k, nmod):
    """Returns (status, beta, [moduli])."""
    beta = ctypes.c_int32()
    mods = (ctypes.c_int32 * max(1, int(nmod)))()
    rc = lib().cosma_ozaki2_params(int(k), int(nmod), ctypes.byref(beta), mods)
    return rc, beta.value, list(mods)[:max(0, int(nmod))]


def cosma_tile_count(dtype) -> int:
    return lib().cosma_tile_count(_dtype(dtype))


def cosma_tile_shape(dtype, tile_id):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = lib().cosma_tile_shape(_dtype(dtype), tile_id, ctypes.byref(a), ctypes.byref(b),
                                ctypes.byref(c))
    return rc, (a.value, b.value, c.value)


def cosma_device_query():
    f = cosma_device_facts()
    rc = lib().cosma_device_query(ctypes.byref(f))
    return rc, f


def cosma_thm1_bound(m, n, k, S) -> float:
    return lib().cosma_thm1_bound(float(m), float(n), float(k), float(S))


def cosma_seq_schedule(S):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().cosma_seq_schedule(int(S), ctypes.byref(a), ctypes.byref(b))
    return rc, a.value, b.value


def cosma_par_schedule(m, n, k, p, S):
    a, b = ctypes.c_double(), ctypes.c_double()
    rc = lib().cosma_par_schedule(float(m), float(n), float(k), float(p), float(S),
                                  ctypes.byref(a), ctypes.byref(b))
    return rc, a.value, b.value


def cosma_fit_ranks(m, n, k, p, delta):
    g = (ctypes.c_int64 * 3)()
    used = ctypes.c_int64()
    rc = lib().cosma_fit_ranks(m, n, k, p, float(delta), g, ctypes.byref(used))
    return rc, (g[0], g[1], g[2]), used.value


def cosma_io_count(m, n, k, tile_m, tile_n, kc, p_k, beta_nonzero=False) -> float:
    return lib().cosma_io_count(m, n, k, tile_m, tile_n, kc, p_k, 1 if beta_nonzero else 0)


def cosma_workspace_size(m, n, k, dtype):
    b = ctypes.c_size_t()
    rc = lib().cosma_workspace_size(m, n, k, _dtype(dtype), ctypes.byref(b))
    return rc, b.value


def cosma_set_workspace(ptr, nbytes, stream=None) -> int:
    return lib().cosma_set_workspace(_ptr(ptr), int(nbytes), None if stream is None else _stream(stream))


# ------------------------------------------------------------ torch helpers
_workspace = {}


def check(rc: int, what: str = "") -> None:
    if rc != COSMA_OK:
        raise CosmaError(rc, what)


def ensure_workspace(nbytes: int, device=None):
    """Register a device workspace of at least nbytes (a torch uint8 buffer
    kept alive here), growing the previous one if needed."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    cur = _workspace.get(dev.index)
    if cur is not None and cur.numel() >= nbytes:
        return cur
    if nbytes == 0:
        return cur
    torch.cuda.synchronize(dev)
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        check(cosma_set_workspace(buf, buf.numel()), "cosma_set_workspace")
    _workspace[dev.index] = buf
    return buf


def gemm(A, B, C, alpha=1.0, beta=0.0, dtype=None, stream=None, plan=None):
    """C = alpha*A@B + beta*C on row-major torch tensors (unit column stride).

    dtype defaults from the tensors: float64 -> "f64", float32 -> "f32".
    """
    import torch
    if dtype is None:
        dtype = "f64" if A.dtype == torch.float64 else "f32"
    d = _dtype(dtype)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    for t in (A, B, C):
        if t.dim() == 2 and t.shape[1] > 1 and t.stride(1) != 1:
            raise ValueError("operands must be row-major with unit column stride")
    lda = A.stride(0) if m > 1 else max(1, k)
    ldb = B.stride(0) if k > 1 else max(1, n)
    ldc = C.stride(0) if m > 1 else max(1, n)
    if plan is None:
        rc, ws = cosma_workspace_size(m, n, k, d)
    else:
        rc, ws = COSMA_OK, plan.workspace_bytes
    check(rc, "cosma_workspace_size")
    if ws:
        ensure_workspace(ws, C.device)
    if plan is None:
        rc = cosma_gemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, d, stream)
    else:
        rc = cosma_gemm_planned(plan, alpha, A, lda, B, ldb, beta, C, ldc, stream)
    check(rc, "cosma_gemm")
    return C
