"""CPU oracle for the xyz interaction search -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never loads it and shares no code with
it.  The arithmetic lives in ``xyz_oracle.c`` (plain C, built into
``liboracle.so`` by ``oracle.build.build_oracle``); this module marshals numpy
arrays in and out and holds the paper's closed forms (``theory``).

Every function cites the passage of the paper it follows.  Parity of the
sampler against the paper is unpinned (the paper's R code uses its own RNG);
the sampler is pinned to SplitMix64's published outputs instead.
"""
from __future__ import annotations

import ctypes
import os
import numpy as np

from . import theory  # noqa: F401  (closed forms, eqs. (8), (9), (11), (15))

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

PAIR_DTYPE = np.dtype([("j", np.int32), ("k", np.int32), ("s", np.int64), ("value", np.float64),
                       ("stat", np.float64), ("first_rep", np.int32), ("hits", np.int32)])
REP_DTYPE = np.dtype([("candidates", np.int64), ("passed", np.int64), ("fresh", np.int64),
                      ("cmask", np.uint64), ("max_bucket", np.int32), ("pad", np.int32)])

_lib = None


def lib():
    """Load liboracle.so (building it first when it is missing and gcc is present)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build_oracle
            build_oracle()
        L = ctypes.CDLL(LIB_PATH)
        L.xo_splitmix64.restype = ctypes.c_uint64
        L.xo_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.xo_draw_rows.restype = ctypes.c_int
        L.xo_draw_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64,
                                   ctypes.c_int, ctypes.c_void_p]
        L.xo_pair_s.restype = ctypes.c_int64
        L.xo_pair_s.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.xo_pair_v.restype = ctypes.c_double
        L.xo_pair_v.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.xo_search.restype = ctypes.c_int
        L.xo_search.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.xo_search_ex.restype = ctypes.c_int
        L.xo_search_ex.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_double, ctypes.POINTER(ctypes.c_void_p),
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.xo_brute.restype = ctypes.c_int
        L.xo_brute.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64)]
        L.xo_free.restype = None
        L.xo_free.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _x_arg(XT):
    """X in column-major order: XT is (p, n).  int8 +-1 -> kind 0, else binary64 -> kind 1."""
    XT = np.asarray(XT)
    if XT.dtype == np.int8:
        return np.ascontiguousarray(XT), 0
    return np.ascontiguousarray(XT, dtype=np.float64), 1


def _y_arg(Y):
    Y = np.asarray(Y)
    if Y.dtype == np.int8:
        return np.ascontiguousarray(Y), 0
    return np.ascontiguousarray(Y, dtype=np.float64), 1


def splitmix64(seed: int, k: int) -> int:
    """Output number k (k >= 1) of SplitMix64 seeded with ``seed``."""
    return int(lib().xo_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))


def draw_rows(n: int, seed: int, l: int, m: int, Y=None) -> np.ndarray:
    """Row indices of repetition l (eq. (6), i.i.d. with replacement).

    Uniform when Y is None or +-1 int8; |Y|-weighted (Section 3.1) for real Y.
    """
    out = np.empty(max(m, 1), dtype=np.int32)
    yp = None
    if Y is not None and np.asarray(Y).dtype != np.int8:
        Yd = np.ascontiguousarray(Y, dtype=np.float64)
        yp = Yd.ctypes.data
    rc = lib().xo_draw_rows(yp, n, seed & (2**64 - 1), l, m, out.ctypes.data)
    if rc != 0:
        raise OracleError(f"xo_draw_rows failed ({rc})")
    return out[:m]


def pair_value(XT, Y, j: int, k: int):
    """Y^T (X_j o X_k) (eq. (1)): exact int for +-1 data, binary64 ascending-i sum otherwise."""
    XT_, xk = _x_arg(XT)
    Y_, yk = _y_arg(Y)
    n = XT_.shape[1]
    if xk == 0 and yk == 0:
        return int(lib().xo_pair_s(XT_.ctypes.data, Y_.ctypes.data, n, j, k))
    Xd = XT_ if xk == 1 else XT_.astype(np.float64)
    Yd = Y_ if yk == 1 else Y_.astype(np.float64)
    return float(lib().xo_pair_v(Xd.ctypes.data, Yd.ctypes.data, n, j, k))


def _take_pairs(ptr, npairs):
    if npairs == 0:
        if ptr:
            lib().xo_free(ptr)
        return np.zeros(0, dtype=PAIR_DTYPE)
    buf = (ctypes.c_char * (npairs * PAIR_DTYPE.itemsize)).from_address(ptr)
    arr = np.frombuffer(bytes(buf), dtype=PAIR_DTYPE).copy()
    lib().xo_free(ptr)
    return arr


def search(XT, Y, m: int, L: int, kappa: float, seed: int = 0, two_sided: bool = False,
           rep_offset: int = 0, rows=None, unbiased: bool = False, cap: float = 0.0):
    """Algorithm 2 run by the oracle.  Returns (pairs, reps) structured arrays.

    XT: (p, n) int8 +-1 or real; Y: (n,) int8 +-1 or real.  rows: optional
    (L, m) int32 table of row indices replacing the sampler.  unbiased (real X
    only): the unbiased transform of Section 3.2 with row scaling instead of
    the sign transform.  cap (unbiased only; 0: none): entries are capped at
    +-cap, rounded to float32, before the transform (Section 3.2's remark on
    capping).
    """
    XT_, xk = _x_arg(XT)
    Y_, yk = _y_arg(Y)
    p, n = XT_.shape
    reps = np.zeros(max(L, 1), dtype=REP_DTYPE)
    rp = None
    if rows is not None:
        rows_ = np.ascontiguousarray(rows, dtype=np.int32).reshape(L, m)
        rp = rows_.ctypes.data
    out = ctypes.c_void_p()
    cnt = ctypes.c_int64()
    rc = lib().xo_search_ex(XT_.ctypes.data, xk, Y_.ctypes.data, yk, n, p, m, L, float(kappa),
                            seed & (2**64 - 1), int(bool(two_sided)), rep_offset, rp, int(bool(unbiased)),
                            float(cap), ctypes.byref(out), ctypes.byref(cnt), reps.ctypes.data)
    if rc != 0:
        raise OracleError(f"xo_search failed ({rc})")
    return _take_pairs(out.value, cnt.value), reps[:L]


def brute(XT, Y, kappa: float, two_sided: bool = False):
    """The plain definition of eq. (1): every pair j < k with Y^T(X_j o X_k)/n > kappa."""
    XT_, xk = _x_arg(XT)
    Y_, yk = _y_arg(Y)
    p, n = XT_.shape
    out = ctypes.c_void_p()
    cnt = ctypes.c_int64()
    rc = lib().xo_brute(XT_.ctypes.data, xk, Y_.ctypes.data, yk, n, p, float(kappa),
                        int(bool(two_sided)), ctypes.byref(out), ctypes.byref(cnt))
    if rc != 0:
        raise OracleError(f"xo_brute failed ({rc})")
    return _take_pairs(out.value, cnt.value)


from . import dense  # noqa: E402,F401  (Algorithm 1 with dense projections)
