"""Python binding of libxyz, the gfx950 implementation of the xyz interaction search.

Argument marshalling only: every function below forwards to the C ABI of
``include/xyz.h`` (same names) through ctypes, and every step of the search
runs in the library's HIP kernels.  The library must be built in-tree
(``paper_1610_05108_amd/libxyz.so``); importing a function that needs it
raises when it is missing -- there is no CPU fallback.

PyTorch is used only as plumbing: a CUDA (HIP) tensor's ``data_ptr()`` is
passed as a device pointer and the current torch stream as the HIP stream.
numpy arrays are passed as host pointers.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxyz.so")

XYZ_OK, XYZ_EINVAL, XYZ_ENOMEM, XYZ_EDEVICE, XYZ_EAGAIN, XYZ_ECANCELED, XYZ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
XYZ_EINTERNAL = -7
XYZ_MEM_HOST, XYZ_MEM_DEVICE = 0, 1
XYZ_X_I8_PM1, XYZ_X_BITS, XYZ_X_F32, XYZ_X_I8_PM1_ROWMAJOR = 0, 1, 2, 3
XYZ_Y_I8_PM1, XYZ_Y_F32, XYZ_Y_F64 = 0, 1, 2
XYZ_TWO_SIDED, XYZ_PROFILE, XYZ_EXACT, XYZ_UNBIASED, XYZ_ROUTE = 1, 2, 4, 8, 16
XYZ_SERVE_SEED = 0x9E3779B97F4A7C15
XYZ_MAX_M = 30

PAIR_DTYPE = np.dtype([("j", np.int32), ("k", np.int32), ("s", np.int64), ("value", np.float64),
                       ("stat", np.float64), ("first_rep", np.int32), ("hits", np.int32)])
REP_DTYPE = np.dtype([("candidates", np.int64), ("passed", np.int64), ("fresh", np.int64),
                      ("cmask", np.uint64), ("max_bucket", np.int32), ("reserved", np.int32)])

EXPORTS = [
    "xyz_version", "xyz_last_error", "xyz_init", "xyz_fini", "xyz_ctx_bytes", "xyz_x_create", "xyz_x_destroy",
    "xyz_x_n", "xyz_x_p", "xyz_search", "xyz_search_batch", "xyz_search_noalloc", "xyz_bruteforce", "xyz_dense_search", "xyz_result_npairs",
    "xyz_result_pairs", "xyz_result_nreps", "xyz_result_reps", "xyz_result_timing", "xyz_result_route",
    "xyz_result_free", "xyz_smin",
    "xyz_eta", "xyz_tau_dense", "xyz_eta_dense", "xyz_L_for", "xyz_m_for_L", "xyz_mstar",
    "xyz_sample_strengths", "xyz_plan",
    "xyz_serve_start", "xyz_serve_submit", "xyz_serve_poll", "xyz_serve_wait", "xyz_serve_cancel",
    "xyz_serve_stats_get", "xyz_serve_stop", "xyz_autotune",
]
XYZ_PLAN_XYZ, XYZ_PLAN_BRUTE = 0, 1


class XyzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libxyz error {code}: {msg}")
        self.code = code


class xyz_params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("L", ctypes.c_int32), ("kappa", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("rep_offset", ctypes.c_int32),
                ("rows", ctypes.c_void_p), ("cap", ctypes.c_double)]


class xyz_timing(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in
                ("total_ms", "pack_ms", "sample_ms", "hash_ms", "bucket_ms", "tiles_ms", "verify_ms",
                 "dedup_ms", "brute_ms")] + [("verify_launches", ctypes.c_int64), ("candidates", ctypes.c_int64),
                                             ("tiles", ctypes.c_int64), ("big_ms", ctypes.c_double),
                                             ("big_launches", ctypes.c_int64), ("big_candidates", ctypes.c_int64),
                                             ("chunks", ctypes.c_int64), ("host_syncs", ctypes.c_int64)]


class xyz_route(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("m", ctypes.c_int32), ("L", ctypes.c_int32), ("routed", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("predicted_ms", ctypes.c_double), ("alternative_ms", ctypes.c_double)]


class xyz_tuning(ctypes.Structure):
    _fields_ = [("chunk_gib", ctypes.c_double), ("verify_wg_per_cu", ctypes.c_int32),
                ("big_wg_per_cu", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("variants", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class xyz_plan_info(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("m", ctypes.c_int32), ("L", ctypes.c_int32), ("mstar", ctypes.c_int32),
                ("predicted_ms", ctypes.c_double), ("predicted_recall", ctypes.c_double),
                ("expected_candidates", ctypes.c_double), ("brute_ms", ctypes.c_double)]


class xyz_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("max_batch", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("inflight", ctypes.c_int32), ("bytes_inflight", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("bytes_held", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libxyz.so.  Raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    try:  # load torch's HIP runtime first so that the process holds a single one
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "xyz_version": (ctypes.c_char_p, []),
        "xyz_last_error": (ctypes.c_char_p, []),
        "xyz_init": (I32, [ctypes.c_int, U64, ctypes.POINTER(P)]),
        "xyz_fini": (None, [P]),
        "xyz_ctx_bytes": (U64, [P]),
        "xyz_x_create": (I32, [P, P, ctypes.c_int, ctypes.c_int, I64, I64, I64, P, ctypes.POINTER(P)]),
        "xyz_x_destroy": (None, [P]),
        "xyz_x_n": (I64, [P]),
        "xyz_x_p": (I64, [P]),
        "xyz_search": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(xyz_params), P, ctypes.POINTER(P)]),
        "xyz_search_batch": (I32, [P, P, I32, ctypes.POINTER(P), ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(xyz_params), P, ctypes.POINTER(P)]),
        "xyz_search_noalloc": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(xyz_params), P, P, I64,
                                     ctypes.POINTER(I64), P]),
        "xyz_bruteforce": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, D, U32, P, I64, P, I64, P, ctypes.POINTER(P)]),
        "xyz_autotune": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(xyz_params), P, ctypes.c_char_p,
                               ctypes.POINTER(xyz_tuning)]),
        "xyz_dense_search": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, P, I32, I64, D, I32, U32, P,
                                   ctypes.POINTER(P)]),
        "xyz_result_npairs": (I64, [P]),
        "xyz_result_pairs": (P, [P]),
        "xyz_result_nreps": (I32, [P]),
        "xyz_result_reps": (P, [P]),
        "xyz_result_timing": (ctypes.POINTER(xyz_timing), [P]),
        "xyz_result_route": (I32, [P, ctypes.POINTER(xyz_route)]),
        "xyz_result_free": (None, [P]),
        "xyz_smin": (I64, [I64, D, ctypes.c_int]),
        "xyz_eta": (D, [D, I32, I64]),
        "xyz_tau_dense": (D, [I64, I64, D]),
        "xyz_eta_dense": (D, [D, I64]),
        "xyz_L_for": (I64, [D, D]),
        "xyz_m_for_L": (I32, [D, I64, D, I32]),
        "xyz_mstar": (I32, [D, I64, I64, P, I64, D, I32]),
        "xyz_sample_strengths": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, I64, U64, P, P]),
        "xyz_plan": (I32, [P, P, P, ctypes.c_int, ctypes.c_int, D, D, D, U32, P, ctypes.POINTER(xyz_plan_info)]),
        "xyz_serve_start": (I32, [P, U64, I32, I32, ctypes.POINTER(P)]),
        "xyz_serve_submit": (I32, [P, P, P, ctypes.c_int, ctypes.POINTER(xyz_params), ctypes.POINTER(U64)]),
        "xyz_serve_poll": (I32, [P, U64, ctypes.POINTER(P)]),
        "xyz_serve_wait": (I32, [P, U64, ctypes.POINTER(P)]),
        "xyz_serve_cancel": (I32, [P, U64]),
        "xyz_serve_stats_get": (I32, [P, ctypes.POINTER(xyz_serve_stats)]),
        "xyz_serve_stop": (I32, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code: int):
    if code != XYZ_OK:
        raise XyzError(code, (lib().xyz_last_error() or b"").decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """(pointer, memory kind, keep-alive object) of a numpy array or torch tensor."""
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (XYZ_MEM_DEVICE if a.is_cuda else XYZ_MEM_HOST), a
    arr = np.ascontiguousarray(a)
    return arr.ctypes.data, XYZ_MEM_HOST, arr


def _stream(stream, *tensors):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    for t in tensors:
        if _is_torch(t) and t.is_cuda:
            import torch
            return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)
    return ctypes.c_void_p(0)


def _x_format(a) -> int:
    dt = str(a.dtype)
    if dt.endswith("int8"):
        return XYZ_X_I8_PM1
    if dt.endswith("uint64") or dt.endswith("int64"):
        return XYZ_X_BITS
    if dt.endswith("float32"):
        return XYZ_X_F32
    raise ValueError(f"unsupported X dtype {dt}")


def _y_format(a) -> int:
    dt = str(a.dtype)
    if dt.endswith("int8"):
        return XYZ_Y_I8_PM1
    if dt.endswith("float32"):
        return XYZ_Y_F32
    if dt.endswith("float64"):
        return XYZ_Y_F64
    raise ValueError(f"unsupported Y dtype {dt}")


# ------------------------------------------------------------- C-ABI names --

def xyz_version() -> str:
    return lib().xyz_version().decode()


def xyz_smin(n: int, kappa: float, two_sided: bool = False) -> int:
    return int(lib().xyz_smin(n, float(kappa), int(bool(two_sided))))


def xyz_init(device: int = 0, hbm_budget_bytes: int = 0):
    h = ctypes.c_void_p()
    _check(lib().xyz_init(device, hbm_budget_bytes, ctypes.byref(h)))
    return h


def xyz_fini(ctx) -> None:
    lib().xyz_fini(ctx)


def xyz_ctx_bytes(ctx) -> int:
    return int(lib().xyz_ctx_bytes(ctx))


def xyz_x_create(ctx, XT, n: int | None = None, stream=None, row_major: bool = False):
    """Make X resident.  XT is X in column-major order, shape (p, n) for int8 +-1 or
    float32, or (p, ceil(n/64)) uint64 packed bits (then n must be given).  With
    row_major, XT is X itself in row-major order: int8 +-1 of shape (n, p)."""
    fmt = _x_format(XT)
    p = int(XT.shape[0])
    if row_major:
        if fmt != XYZ_X_I8_PM1 or XT.ndim != 2:
            raise ValueError("row-major X must be a 2-D int8 array of shape (n, p)")
        fmt, n, p, ld = XYZ_X_I8_PM1_ROWMAJOR, int(XT.shape[0]), int(XT.shape[1]), int(XT.shape[1])
    elif fmt == XYZ_X_BITS:
        if n is None:
            raise ValueError("n is required for packed bits")
        ld = int(XT.shape[1])
    else:
        n = int(XT.shape[1]) if n is None else n
        ld = int(XT.shape[1])
    ptr, mem, keep = _ptr(XT)
    h = ctypes.c_void_p()
    _check(lib().xyz_x_create(ctx, ptr, fmt, mem, n, p, ld, _stream(stream, XT), ctypes.byref(h)))
    del keep
    return h


def xyz_x_destroy(x) -> None:
    lib().xyz_x_destroy(x)


def xyz_x_n(x) -> int:
    return int(lib().xyz_x_n(x))


def xyz_x_p(x) -> int:
    return int(lib().xyz_x_p(x))


def _check_y(x, Y):
    """The C side reads n entries of Y: refuse a response of another length."""
    n = xyz_x_n(x)
    size = int(Y.numel()) if _is_torch(Y) else int(np.size(Y))
    if size != n:
        raise ValueError(f"Y has {size} entries; X has n = {n} rows")


def _params(m, L, kappa, seed, two_sided, rep_offset, rows, profile, unbiased=False, cap=0.0):
    prm = xyz_params()
    prm.cap = float(cap)
    prm.m, prm.L, prm.kappa, prm.seed = int(m), int(L), float(kappa), int(seed) & (2 ** 64 - 1)
    prm.flags = ((XYZ_TWO_SIDED if two_sided else 0) | (XYZ_PROFILE if profile else 0) |
                 (XYZ_UNBIASED if unbiased else 0))
    prm.rep_offset = int(rep_offset)
    keep = None
    if rows is not None:
        keep = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1)
        if keep.size != int(L) * int(m):
            raise ValueError("rows must hold L*m entries")
        prm.rows = keep.ctypes.data
    return prm, keep


def _take_result(h):
    L = lib()
    npairs = int(L.xyz_result_npairs(h))
    pairs = np.zeros(npairs, dtype=PAIR_DTYPE)
    if npairs:
        ctypes.memmove(pairs.ctypes.data, L.xyz_result_pairs(h), npairs * PAIR_DTYPE.itemsize)
    nreps = int(L.xyz_result_nreps(h))
    reps = np.zeros(nreps, dtype=REP_DTYPE)
    if nreps:
        ctypes.memmove(reps.ctypes.data, L.xyz_result_reps(h), nreps * REP_DTYPE.itemsize)
    t = L.xyz_result_timing(h).contents
    timing = {name: getattr(t, name) for name, _ in xyz_timing._fields_}
    rt = xyz_route()
    L.xyz_result_route(h, ctypes.byref(rt))
    route = {name: getattr(rt, name) for name, _ in xyz_route._fields_}
    L.xyz_result_free(h)
    return {"pairs": pairs, "reps": reps, "timing": timing, "route": route}


def xyz_search(ctx, x, Y, m: int, L: int, kappa: float, seed: int = 0, two_sided: bool = False,
               rep_offset: int = 0, rows=None, profile: bool = False, stream=None, unbiased: bool = False,
               cap: float = 0.0):
    """Algorithm 2 on resident X.  Returns {'pairs', 'reps', 'timing'}.  unbiased:
    hash float32 X with the unbiased transform of Section 3.2 (XYZ_UNBIASED);
    cap > 0 caps the entries at +-cap first (xyz_params.cap)."""
    _check_y(x, Y)
    prm, keep_rows = _params(m, L, kappa, seed, two_sided, rep_offset, rows, profile, unbiased, cap)
    ptr, mem, keep = _ptr(Y)
    h = ctypes.c_void_p()
    _check(lib().xyz_search(ctx, x, ptr, _y_format(Y), mem, ctypes.byref(prm), _stream(stream, Y), ctypes.byref(h)))
    del keep, keep_rows
    return _take_result(h)


def xyz_search_batch(ctx, x, Ys, params: list, stream=None):
    """Several searches on one X; params[q] is a dict of xyz_search keywords."""
    nY = len(Ys)
    if nY == 0:
        return []
    fmts = {_y_format(Y) for Y in Ys}
    if len(fmts) != 1:
        raise ValueError("all Y must share one format")
    ptrs, keeps, mems = [], [], set()
    for Y in Ys:
        _check_y(x, Y)
        ptr, mem, keep = _ptr(Y)
        ptrs.append(ptr)
        keeps.append(keep)
        mems.add(mem)
    if len(mems) != 1:
        raise ValueError("all Y must live in the same memory")
    arr = (xyz_params * nY)()
    keep_rows = []
    for q, kw in enumerate(params):
        prm, kr = _params(kw["m"], kw["L"], kw["kappa"], kw.get("seed", 0), kw.get("two_sided", False),
                          kw.get("rep_offset", 0), kw.get("rows"), kw.get("profile", False),
                          kw.get("unbiased", False), kw.get("cap", 0.0))
        arr[q] = prm
        keep_rows.append(kr)
    yp = (ctypes.c_void_p * nY)(*ptrs)
    outs = (ctypes.c_void_p * nY)()
    _check(lib().xyz_search_batch(ctx, x, nY, yp, fmts.pop(), mems.pop(), arr, _stream(stream, *Ys), outs))
    del keeps, keep_rows
    return [_take_result(outs[q]) for q in range(nY)]


def xyz_search_noalloc(ctx, x, Y, m: int, L: int, kappa: float, seed: int = 0, two_sided: bool = False,
                       rep_offset: int = 0, rows=None, stream=None, unbiased: bool = False, pairs_cap: int = 1 << 16,
                       cap: float = 0.0):
    """xyz_search through the entry point that allocates no memory (workspaces in the library's
    static device scratch).  Returns {'pairs', 'reps'}; raises XyzError (code XYZ_ENOMEM, with
    'npairs' set) when more than pairs_cap pairs are found."""
    if int(L) < 1:
        raise ValueError("L must be >= 1")
    _check_y(x, Y)
    prm, keep_rows = _params(m, L, kappa, seed, two_sided, rep_offset, rows, False, unbiased, cap)
    ptr, mem, keep = _ptr(Y)
    pairs = np.zeros(max(int(pairs_cap), 1), dtype=PAIR_DTYPE)
    reps = np.zeros(int(L), dtype=REP_DTYPE)
    npairs = ctypes.c_int64(0)
    rc = lib().xyz_search_noalloc(ctx, x, ptr, _y_format(Y), mem, ctypes.byref(prm), _stream(stream, Y),
                                  pairs.ctypes.data, int(pairs_cap), ctypes.byref(npairs), reps.ctypes.data)
    del keep, keep_rows
    if rc != XYZ_OK:
        err = XyzError(rc, (lib().xyz_last_error() or b"").decode())
        err.npairs = int(npairs.value)
        raise err
    return {"pairs": pairs[:int(npairs.value)].copy(), "reps": reps}


def xyz_autotune(ctx, x, Y, m: int, L: int, kappa: float, seed: int = 0, two_sided: bool = False,
                 unbiased: bool = False, cap: float = 0.0, cache_path=None, stream=None):
    """Time the search's launch shapes once (xyz_autotune) and keep the fastest for later searches of
    the same shape in the context; cache_path: text file of tuned shapes read before timing and
    updated after.  Returns the choice as a dict (from_cache = 1 when nothing was timed)."""
    _check_y(x, Y)
    prm, keep_rows = _params(m, L, kappa, seed, two_sided, 0, None, False, unbiased, cap)
    ptr, mem, keep = _ptr(Y)
    out = xyz_tuning()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().xyz_autotune(ctx, x, ptr, _y_format(Y), mem, ctypes.byref(prm), _stream(stream, Y), path,
                              ctypes.byref(out)))
    del keep, keep_rows
    return {name: getattr(out, name) for name, _ in xyz_tuning._fields_}


def xyz_dense_search(ctx, x, Y, R, tau: int, kappa: float, rep_offset: int = 0, profile: bool = False,
                     stream=None):
    """Algorithm 1 with dense projections: R is (L, n) int32 (one projection vector
    per repetition, sum |R_l| < 2^31), tau the close-pairs threshold on R's grid.
    Returns {'pairs', 'reps', 'timing'} as xyz_search."""
    R0 = np.asarray(R)
    if R0.ndim != 2 or R0.shape[1] != xyz_x_n(x):
        raise ValueError(f"R must be (L, n) with n = {xyz_x_n(x)}; got shape {R0.shape}")
    if R0.size and (not np.issubdtype(R0.dtype, np.integer) or R0.min() < -(2 ** 31 - 1) or R0.max() > 2 ** 31 - 1):
        raise ValueError("R must hold integers of magnitude below 2^31")
    _check_y(x, Y)
    Rv = np.ascontiguousarray(R0, dtype=np.int32)
    ptr, mem, keep = _ptr(Y)
    h = ctypes.c_void_p()
    _check(lib().xyz_dense_search(ctx, x, ptr, _y_format(Y), mem, Rv.ctypes.data, Rv.shape[0], int(tau),
                                  float(kappa), int(rep_offset), XYZ_PROFILE if profile else 0,
                                  _stream(stream, Y), ctypes.byref(h)))
    del keep
    return _take_result(h)


def xyz_bruteforce(ctx, x, Y, kappa: float, colsA=None, colsB=None, two_sided: bool = False,
                   profile: bool = False, stream=None):
    """Exact eq. (1) over colsA x colsB (all columns when None)."""
    _check_y(x, Y)
    ptr, mem, keep = _ptr(Y)
    a = None if colsA is None else np.ascontiguousarray(colsA, dtype=np.int32)
    b = None if colsB is None else np.ascontiguousarray(colsB, dtype=np.int32)
    flags = (XYZ_TWO_SIDED if two_sided else 0) | (XYZ_PROFILE if profile else 0)
    h = ctypes.c_void_p()
    _check(lib().xyz_bruteforce(ctx, x, ptr, _y_format(Y), mem, float(kappa), flags,
                                None if a is None else a.ctypes.data, 0 if a is None else a.size,
                                None if b is None else b.ctypes.data, 0 if b is None else b.size,
                                _stream(stream, Y), ctypes.byref(h)))
    del keep
    return _take_result(h)


def xyz_eta(gamma: float, m: int, L: int) -> float:
    return float(lib().xyz_eta(float(gamma), int(m), int(L)))


def xyz_tau_dense(p: int, n: int, sd: float = 1.0) -> float:
    return float(lib().xyz_tau_dense(int(p), int(n), float(sd)))


def xyz_eta_dense(gamma: float, p: int) -> float:
    return float(lib().xyz_eta_dense(float(gamma), int(p)))


def xyz_L_for(eta: float, beta: float) -> int:
    return int(lib().xyz_L_for(float(eta), float(beta)))


def xyz_m_for_L(gamma: float, L: int, eta: float, m_max: int = XYZ_MAX_M) -> int:
    return int(lib().xyz_m_for_L(float(gamma), int(L), float(eta), int(m_max)))


def xyz_mstar(gamma: float, n: int, p: int, gammas, total_pairs: float, m_max: int = 64) -> int:
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    return int(lib().xyz_mstar(float(gamma), int(n), int(p), g.ctypes.data, g.size, float(total_pairs), int(m_max)))


def xyz_sample_strengths(ctx, x, Y, npairs: int, seed: int = 0, stream=None) -> np.ndarray:
    _check_y(x, Y)
    out = np.zeros(int(npairs), dtype=np.float64)
    ptr, mem, keep = _ptr(Y)
    _check(lib().xyz_sample_strengths(ctx, x, ptr, _y_format(Y), mem, int(npairs), int(seed) & (2 ** 64 - 1),
                                      _stream(stream, Y), out.ctypes.data))
    del keep
    return out


def xyz_plan(ctx, x, Y, kappa: float, gamma_target: float, eta_target: float = 0.95, two_sided: bool = False,
             stream=None) -> dict:
    _check_y(x, Y)
    info = xyz_plan_info()
    ptr, mem, keep = _ptr(Y)
    _check(lib().xyz_plan(ctx, x, ptr, _y_format(Y), mem, float(kappa), float(gamma_target), float(eta_target),
                          XYZ_TWO_SIDED if two_sided else 0, _stream(stream, Y), ctypes.byref(info)))
    del keep
    return {name: getattr(info, name) for name, _ in xyz_plan_info._fields_}


def xyz_serve_start(ctx, hbm_budget_bytes: int = 0, workers: int = 2, max_batch: int = 64):
    h = ctypes.c_void_p()
    _check(lib().xyz_serve_start(ctx, int(hbm_budget_bytes), int(workers), int(max_batch), ctypes.byref(h)))
    return h


def xyz_serve_submit(server, x, Y, m: int = 0, L: int = 1, kappa: float = 0.0, seed: int = 0,
                     two_sided: bool = False, rep_offset: int = 0, rows=None, exact: bool = False,
                     route: bool = False) -> int:
    """Queue a search (Y is host memory: numpy array or CPU tensor); returns the ticket.
    exact=True asks for the exact search of eq. (1) (m, L, seed, rows ignored); route=True lets the
    server choose between the exact search and xyz with this L (XYZ_ROUTE: m, seed, rows ignored)."""
    if _is_torch(Y) and Y.is_cuda:
        raise ValueError("xyz_serve_submit takes Y in host memory")
    _check_y(x, Y)
    prm, keep_rows = _params(m, L, kappa, seed, two_sided, rep_offset, None if (exact or route) else rows, False)
    if exact:
        prm.flags |= XYZ_EXACT
    if route:
        prm.flags |= XYZ_ROUTE
    ptr, _, keep = _ptr(Y)
    t = ctypes.c_uint64()
    _check(lib().xyz_serve_submit(server, x, ptr, _y_format(Y), ctypes.byref(prm), ctypes.byref(t)))
    del keep, keep_rows
    return int(t.value)


def xyz_serve_poll(server, ticket: int):
    """None while the request is pending, else its result dict (raises on error / cancellation)."""
    h = ctypes.c_void_p()
    rc = lib().xyz_serve_poll(server, int(ticket), ctypes.byref(h))
    if rc == XYZ_EAGAIN:
        return None
    _check(rc)
    return _take_result(h)


def xyz_serve_wait(server, ticket: int):
    h = ctypes.c_void_p()
    _check(lib().xyz_serve_wait(server, int(ticket), ctypes.byref(h)))
    return _take_result(h)


def xyz_serve_cancel(server, ticket: int) -> bool:
    """True if the request was cancelled (or had finished), False if it is already running."""
    rc = lib().xyz_serve_cancel(server, int(ticket))
    if rc == XYZ_EAGAIN:
        return False
    _check(rc)
    return True


def xyz_serve_stats_get(server) -> dict:
    st = xyz_serve_stats()
    _check(lib().xyz_serve_stats_get(server, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in xyz_serve_stats._fields_}


def xyz_serve_stop(server) -> None:
    _check(lib().xyz_serve_stop(server))


class Context:
    """Convenience owner of a context and its resident matrices."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.h = xyz_init(device, hbm_budget_bytes)
        self._xs = []

    def x_create(self, XT, n=None, stream=None, row_major=False):
        x = xyz_x_create(self.h, XT, n=n, stream=stream, row_major=row_major)
        self._xs.append(x)
        return x

    def x_destroy(self, x):
        """Free a matrix made by x_create (once: close() no longer frees it)."""
        for q, h in enumerate(self._xs):
            if h == x:
                del self._xs[q]
                xyz_x_destroy(x)
                return
        raise XyzError(XYZ_EINVAL, "matrix not owned by this context")

    def search(self, x, Y, **kw):
        return xyz_search(self.h, x, Y, **kw)

    def search_noalloc(self, x, Y, **kw):
        return xyz_search_noalloc(self.h, x, Y, **kw)

    def autotune(self, x, Y, **kw):
        return xyz_autotune(self.h, x, Y, **kw)

    def search_batch(self, x, Ys, params, stream=None):
        return xyz_search_batch(self.h, x, Ys, params, stream=stream)

    def dense_search(self, x, Y, R, tau, kappa, **kw):
        return xyz_dense_search(self.h, x, Y, R, tau, kappa, **kw)

    def bruteforce(self, x, Y, kappa, **kw):
        return xyz_bruteforce(self.h, x, Y, kappa, **kw)

    def sample_strengths(self, x, Y, npairs, seed=0, stream=None):
        return xyz_sample_strengths(self.h, x, Y, npairs, seed=seed, stream=stream)

    def plan(self, x, Y, kappa, gamma_target, eta_target=0.95, two_sided=False, stream=None):
        return xyz_plan(self.h, x, Y, kappa, gamma_target, eta_target, two_sided=two_sided, stream=stream)

    def close(self):
        for x in self._xs:
            xyz_x_destroy(x)
        self._xs = []
        if self.h:
            xyz_fini(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
