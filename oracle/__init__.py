"""CPU oracle for the longest-overlap-region path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers. It shares no code with the GPU path
(no kernels, headers, helpers or table generators) and imports nothing from
the GPU package; inputs come from the seeded generators, passed in as arrays.

`liboracle.so` (oracle.c) computes every result straight from the
definitions in Section III of the paper:
  * suffix array  -- comparison sort of all suffixes (Table I order);
  * LCP           -- direct comparison of rank-adjacent suffixes (Table IV);
  * ISA           -- inverse permutation (Table III, 1-based there);
  * range minimum -- naive scan, leftmost position (RMQ definition);
  * pair lcp      -- direct comparison of the two suffixes;
  * overlap       -- max LCP across sequences with the lexicographic tie-break,
                     and separately the O(nm) longest-common-substring DP;
  * certificate   -- permutation + adjacent-order + LCP exactness.
`brute.py` holds pure-Python brute force for tiny inputs and `dc3_paper.py`
the three DC3 steps of Section III, used only to pin the paper's worked
examples.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I32 = ctypes.c_int32
    INT = ctypes.c_int
    lib.orc_join.argtypes = [P, P, I32, P]
    lib.orc_join.restype = I64
    lib.orc_sa_u8.argtypes = [P, I64, P, INT]
    lib.orc_sa_u8.restype = INT
    lib.orc_sa_i32.argtypes = [P, I64, P, INT]
    lib.orc_sa_i32.restype = INT
    lib.orc_pair_lcp_u8.argtypes = [P, I64, I64, I64]
    lib.orc_pair_lcp_u8.restype = I64
    lib.orc_lcp_u8.argtypes = [P, I64, P, P, INT]
    lib.orc_lcp_u8.restype = None
    lib.orc_lcp_i32.argtypes = [P, I64, P, P, INT]
    lib.orc_lcp_i32.restype = None
    lib.orc_isa.argtypes = [P, I64, P]
    lib.orc_isa.restype = None
    lib.orc_range_min.argtypes = [P, I64, I64, ctypes.POINTER(I64)]
    lib.orc_range_min.restype = I32
    lib.orc_pair_queries_u8.argtypes = [P, I64, P, P, I64, P]
    lib.orc_pair_queries_u8.restype = None
    lib.orc_overlap.argtypes = [P, P, I64, P, I32, P]
    lib.orc_overlap.restype = INT
    lib.orc_lcs_dp.argtypes = [P, I64, P, I64, P]
    lib.orc_lcs_dp.restype = INT
    lib.orc_certify_u8.argtypes = [P, I64, P, P, INT]
    lib.orc_certify_u8.restype = I64
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _threads(nthreads):
    return nthreads if nthreads else (os.cpu_count() or 1)


def join(concat: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Joined text: sequence j followed by separator 4+j."""
    lib = _load()
    concat = np.ascontiguousarray(concat, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    out = np.empty(int(offsets[-1]) + k, dtype=np.uint8)
    w = lib.orc_join(_ptr(concat), _ptr(offsets), k, _ptr(out))
    if w < 0:
        raise ValueError("base outside 0..3")
    return out


def suffix_array(text: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """Suffix array by comparison sort (uint8 or int32 text)."""
    lib = _load()
    n = text.size
    sa = np.empty(n, dtype=np.int32)
    if text.dtype == np.uint8:
        t = np.ascontiguousarray(text)
        rc = lib.orc_sa_u8(_ptr(t), n, _ptr(sa), _threads(nthreads))
    else:
        t = np.ascontiguousarray(text, dtype=np.int32)
        rc = lib.orc_sa_i32(_ptr(t), n, _ptr(sa), _threads(nthreads))
    if rc:
        raise MemoryError("oracle suffix sort")
    return sa


def lcp(text: np.ndarray, sa: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """LCP[r] = lcp(SA[r-1], SA[r]) by direct comparison; LCP[0] = 0."""
    lib = _load()
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    out = np.empty(sa.size, dtype=np.int32)
    if text.dtype == np.uint8:
        t = np.ascontiguousarray(text)
        lib.orc_lcp_u8(_ptr(t), t.size, _ptr(sa), _ptr(out), _threads(nthreads))
    else:
        t = np.ascontiguousarray(text, dtype=np.int32)
        lib.orc_lcp_i32(_ptr(t), t.size, _ptr(sa), _ptr(out), _threads(nthreads))
    return out


def isa(sa: np.ndarray) -> np.ndarray:
    lib = _load()
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    out = np.empty(sa.size, dtype=np.int32)
    lib.orc_isa(_ptr(sa), sa.size, _ptr(out))
    return out


def pair_lcp(text: np.ndarray, i: int, j: int) -> int:
    lib = _load()
    t = np.ascontiguousarray(text, dtype=np.uint8)
    return int(lib.orc_pair_lcp_u8(_ptr(t), t.size, int(i), int(j)))


def pair_queries(text: np.ndarray, qi: np.ndarray, qj: np.ndarray) -> np.ndarray:
    """lcp of suffix pairs (qi[k], qj[k]) by direct comparison."""
    lib = _load()
    t = np.ascontiguousarray(text, dtype=np.uint8)
    qi = np.ascontiguousarray(qi, dtype=np.int32)
    qj = np.ascontiguousarray(qj, dtype=np.int32)
    out = np.empty(qi.size, dtype=np.int32)
    lib.orc_pair_queries_u8(_ptr(t), t.size, _ptr(qi), _ptr(qj), qi.size, _ptr(out))
    return out


def range_min(a: np.ndarray, lo: int, hi: int):
    """(min a[lo..hi], leftmost argmin), inclusive bounds."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.int32)
    am = ctypes.c_int64(-1)
    v = lib.orc_range_min(_ptr(a), int(lo), int(hi), ctypes.byref(am))
    return int(v), int(am.value)


def overlap(sa: np.ndarray, lcp_arr: np.ndarray, offsets: np.ndarray) -> tuple:
    """(L, seq_p, off_p, seq_q, off_q) from SA and LCP of the joined text."""
    lib = _load()
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    lcp_arr = np.ascontiguousarray(lcp_arr, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    out = np.empty(5, dtype=np.int64)
    if lib.orc_overlap(_ptr(sa), _ptr(lcp_arr), sa.size, _ptr(offsets), offsets.size - 1, _ptr(out)):
        raise MemoryError("oracle overlap")
    return tuple(int(x) for x in out)


def lcs_dp(a: np.ndarray, b: np.ndarray) -> tuple:
    """(length, start in a, start in b) by the O(nm) DP, first maximum in row-major order."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.empty(3, dtype=np.int64)
    if lib.orc_lcs_dp(_ptr(a), a.size, _ptr(b), b.size, _ptr(out)):
        raise MemoryError("oracle dp")
    return tuple(int(x) for x in out)


def certify(text: np.ndarray, sa: np.ndarray, lcp_arr: np.ndarray | None = None,
            nthreads: int | None = None) -> int:
    """-1 if sa (and lcp) are certified exact for text; -2 if sa is not a
    permutation; otherwise the first rank where adjacent order/LCP fails."""
    lib = _load()
    t = np.ascontiguousarray(text, dtype=np.uint8)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    lp = None
    if lcp_arr is not None:
        lcp_arr = np.ascontiguousarray(lcp_arr, dtype=np.int32)
        lp = _ptr(lcp_arr)
    return int(lib.orc_certify_u8(_ptr(t), t.size, _ptr(sa), lp, _threads(nthreads)))
