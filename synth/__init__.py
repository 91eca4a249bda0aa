"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws numbers; it holds none of the matrix-multiplication
arithmetic.  Every value is a pure function of (seed, stream, logical index),
so any sub-block of a matrix can be regenerated on the host without building
the whole matrix, and the device fill kernel in ``fill.hip`` (an independent
implementation of the same definition) produces bit-identical values on the
GPU.

Generator: the splitmix64 output function (Steele, Lea & Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), used as a
counter-based hash::

    mix(z)  : z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
              z ^= z >> 27; z *= 0x94D049BB133111EB
              z ^= z >> 31
    key     = mix((4*seed + stream + 1) * GAMMA)
    h(i)    = mix(key + (i + 1) * GAMMA)          (all arithmetic mod 2^64)

with GAMMA = 0x9E3779B97F4A7C15.  Element (r, c) of a rows x cols matrix uses
the logical index i = r*cols + c, independent of any leading dimension.

Distributions (``dist``):
  UNIFORM_F64  (h >> 11) * 2^-52 - 1            exact binary64 in [-1, 1)
  UNIFORM_F32  (h >> 40) * 2^-23 - 1            exact binary32 in [-1, 1)
  WIDE_F64     s * (1 + ((h >> 11) & (2^52-1)) * 2^-52) * 2^e,
               s = -1 if bit 63 of h else +1, e = (h' mod 41) - 20 where h'
               is the hash of the same index in stream (stream + 8)
  INT_F64 / INT_F32   (h mod (2R+1)) - R, an integer in [-R, R]
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

UNIFORM_F64 = 0
UNIFORM_F32 = 1
WIDE_F64 = 2
INT_F64 = 3
INT_F32 = 4

STREAM_A = 0
STREAM_B = 1
STREAM_C = 2

_F32_DISTS = (UNIFORM_F32, INT_F32)


def dist_dtype(dist: int):
    return np.float32 if dist in _F32_DISTS else np.float64


def mix_int(z: int) -> int:
    """splitmix64 output function on a Python int (reference scalar form)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def key_int(seed: int, stream: int) -> int:
    return mix_int(((4 * seed + stream + 1) * GAMMA) & MASK64)


def hash_int(seed: int, stream: int, i: int) -> int:
    return mix_int((key_int(seed, stream) + (i + 1) * GAMMA) & MASK64)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def hashes(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Vectorised h(seed, stream, idx) for an integer index array."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = np.uint64(key_int(seed, stream))
    with np.errstate(over="ignore"):
        z = key + (idx + np.uint64(1)) * np.uint64(GAMMA)
        return _mix(z)


def values_from_hash(h: np.ndarray, dist: int, param: int = 0,
                     h_exp: np.ndarray | None = None) -> np.ndarray:
    if dist == UNIFORM_F64:
        return (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
    if dist == UNIFORM_F32:
        v = (h >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -23)
        return v - np.float32(1.0)
    if dist == WIDE_F64:
        mant = 1.0 + (h >> np.uint64(11) & np.uint64((1 << 52) - 1)).astype(np.float64) * 2.0 ** -52
        sign = np.where((h >> np.uint64(63)) != 0, -1.0, 1.0)
        e = (h_exp % np.uint64(41)).astype(np.int64) - 20
        return sign * np.ldexp(mant, e)
    if dist in (INT_F64, INT_F32):
        r = int(param)
        if r < 0:
            raise ValueError("integer range must be >= 0")
        v = (h % np.uint64(2 * r + 1)).astype(np.int64) - r
        return v.astype(dist_dtype(dist))
    raise ValueError(f"unknown distribution {dist}")


def gen(rows: int, cols: int, seed: int, stream: int, dist: int, param: int = 0,
        row_idx=None, col_idx=None) -> np.ndarray:
    """Matrix (or the sub-block row_idx x col_idx of it) of a rows x cols matrix."""
    r = np.arange(rows, dtype=np.uint64) if row_idx is None else np.asarray(row_idx, dtype=np.uint64)
    c = np.arange(cols, dtype=np.uint64) if col_idx is None else np.asarray(col_idx, dtype=np.uint64)
    if r.size and int(r.max()) >= rows or c.size and int(c.max()) >= cols:
        raise IndexError("sub-block index outside the matrix")
    idx = r[:, None] * np.uint64(cols) + c[None, :]
    h = hashes(seed, stream, idx)
    h_exp = hashes(seed, stream + 8, idx) if dist == WIDE_F64 else None
    return values_from_hash(h, dist, param, h_exp)


def batch_dims(count: int, seed: int, lo: int = 64, hi: int = 4096) -> np.ndarray:
    """(count, 3) int64 array of (m, n, k), each log-uniform in [lo, hi].

    Dimension d of problem p uses u = (h >> 11) * 2^-53 from stream 16 + d at
    index p and takes floor(lo * (hi/lo)^u), clipped to [lo, hi].
    """
    out = np.empty((count, 3), dtype=np.int64)
    span = np.log2(hi / lo)
    for d in range(3):
        h = hashes(seed, 16 + d, np.arange(count, dtype=np.uint64))
        u = (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        x = np.floor(lo * np.exp2(span * u)).astype(np.int64)
        out[:, d] = np.clip(x, lo, hi)
    return out


def memory_scenarios(S_words: float, p: int):
    """The paper's memory-scaling shapes (section 8, "Selection of
    Benchmarks"; figure captions of section 9) for p processors with S
    words each: "limited memory" keeps p S / I fixed, "extra memory"
    p^(2/3) S / I, with I = mn + mk + nk the input size; here both constants
    are 1.  Shapes: square (n = sqrt(I / 3)); largeK, the RPA water shape
    m = n = 136 w, k = 228 w^2 (section 8's application benchmark); largeM,
    its transpose m = 228 w^2, n = k = 136 w; flat, the rank-256 update with
    k = 256.  Also the square sizes around the switch of eq. optTileShape,
    mnk / p = S^(3/2) (0.75x, 1x, 1.3x).  Returns [(name, (m, n, k))]."""
    import math

    def rpa_w(I):
        lo, hi = 0.01, 1e4
        for _ in range(200):
            w = 0.5 * (lo + hi)
            if 2 * 136 * 228 * w ** 3 + 136 * 136 * w * w > I:
                hi = w
            else:
                lo = w
        return w

    out = []
    for tag, I in (("limited", p * S_words), ("extra", p ** (2.0 / 3.0) * S_words)):
        w = rpa_w(I)
        mm, kk = round(136 * w), round(228 * w * w)
        fl = round(-256 + math.sqrt(256 * 256 + I))
        out += [(f"square {tag}", (round(math.sqrt(I / 3)),) * 3),
                (f"largeK {tag}", (mm, mm, kk)), (f"largeM {tag}", (kk, mm, mm)),
                (f"flat {tag}", (fl, fl, 256))]
    sw = (p * S_words ** 1.5) ** (1.0 / 3.0)
    out += [("optTileShape switch x0.75", (round(0.75 * sw),) * 3),
            ("optTileShape switch", (round(sw),) * 3),
            ("optTileShape switch x1.3", (round(1.3 * sw),) * 3)]
    return out


# ------------------------------------------------------------------ device fill
import ctypes as _ct
import os as _os
import subprocess as _sp

_FILL_SRC = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "fill.hip")
_FILL_LIB = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "libsynth_fill.so")
_fill = None


def build_fill(hipcc: str = "/opt/rocm/bin/hipcc") -> str:
    """Compile the device fill kernel for gfx950 (always recompiles)."""
    tmp = _FILL_LIB + ".tmp%d" % _os.getpid()
    _sp.check_call([hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-o", tmp, _FILL_SRC], stderr=_sp.DEVNULL)
    _os.replace(tmp, _FILL_LIB)
    return _FILL_LIB


def _fill_lib():
    global _fill
    if _fill is None:
        if not _os.path.exists(_FILL_LIB):
            build_fill()
        L = _ct.CDLL(_FILL_LIB)
        L.synth_fill.restype = _ct.c_int
        L.synth_fill.argtypes = [_ct.c_void_p, _ct.c_int64, _ct.c_int64, _ct.c_int64, _ct.c_uint64,
                                 _ct.c_uint32, _ct.c_int, _ct.c_int64, _ct.c_void_p]
        _fill = L
    return _fill


def fill_device(t, seed: int, stream: int, dist: int, param: int = 0, hip_stream=None) -> None:
    """Fill the 2-D torch device tensor t (row-major, unit column stride) with
    the same values gen() gives for a t.shape[0] x t.shape[1] matrix."""
    import torch
    rows, cols = t.shape
    if cols > 1 and t.stride(1) != 1:
        raise ValueError("unit column stride required")
    want = torch.float32 if dist in _F32_DISTS else torch.float64
    if t.dtype != want:
        raise ValueError(f"distribution {dist} fills {want}, got {t.dtype}")
    ld = t.stride(0) if rows > 1 else max(cols, 1)
    s = hip_stream if hip_stream is not None else torch.cuda.current_stream().cuda_stream
    rc = _fill_lib().synth_fill(t.data_ptr(), rows, cols, ld, seed & MASK64, stream, dist, param, s)
    if rc != 0:
        raise RuntimeError(f"synth_fill failed ({rc})")
