"""CPU oracle for Interval Tree Matching -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library and its Python binding never do.

Python side of the oracle: a ctypes binding of ``itm_oracle.c`` (the plain C
matchers: ITM with a literal d-way list intersection, brute force, sort-based
matching) plus small numpy helpers whose every line is a definition from the
paper.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_build.LIB)
                or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        fp = ctypes.POINTER(ctypes.c_float)
        u64pp = ctypes.POINTER(ctypes.POINTER(ctypes.c_uint64))
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_itm.argtypes = [fp, fp, ctypes.c_uint32, fp, fp, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u64pp, u64p]
        L.oracle_itm.restype = ctypes.c_int
        L.oracle_brute.argtypes = [fp, fp, ctypes.c_uint32, fp, fp, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_int, u64pp, u64p]
        L.oracle_brute.restype = ctypes.c_int
        L.oracle_sbm_1d.argtypes = [fp, fp, ctypes.c_uint32, fp, fp, ctypes.c_uint32,
                                    u64pp, u64p]
        L.oracle_sbm_1d.restype = ctypes.c_int
        L.oracle_itm_1d_visits.argtypes = [fp, fp, ctypes.c_uint32, fp, fp,
                                           ctypes.c_uint32, u64p, u32p, u32p]
        L.oracle_itm_1d_visits.restype = ctypes.c_int
        L.oracle_pst_1d.argtypes = [fp, fp, ctypes.c_uint32, fp, fp, ctypes.c_uint32,
                                    u64pp, u64p, u64p, u32p]
        L.oracle_pst_1d.restype = ctypes.c_int
        L.oracle_free.argtypes = [ctypes.c_void_p]
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _take_keys(rc, keys_p, count):
    L = lib()
    if rc != 0:
        raise OracleError(rc)
    K = int(count.value)
    if K == 0:
        if keys_p:
            L.oracle_free(keys_p)
        return np.zeros(0, dtype=np.uint64)
    out = np.ctypeslib.as_array(keys_p, shape=(K,)).copy()
    L.oracle_free(keys_p)
    return out


def _dims(s_lo, u_lo):
    s_lo = np.asarray(s_lo)
    u_lo = np.asarray(u_lo)
    d = s_lo.shape[0] if s_lo.ndim == 2 else 1
    n = s_lo.shape[-1]
    m = u_lo.shape[-1]
    return d, n, m


def itm(s_lo, s_hi, u_lo, u_hi, threads: int = 1, strict: bool = False) -> np.ndarray:
    """Sorted u64 keys (update << 32) | subscription of all intersecting pairs."""
    d, n, m = _dims(s_lo, u_lo)
    a, pa = _f32(s_lo); b, pb = _f32(s_hi); c, pc = _f32(u_lo); e, pe = _f32(u_hi)
    keys = ctypes.POINTER(ctypes.c_uint64)()
    cnt = ctypes.c_uint64(0)
    rc = lib().oracle_itm(pa, pb, n, pc, pe, m, d, int(threads), int(strict),
                          ctypes.byref(keys), ctypes.byref(cnt))
    return _take_keys(rc, keys, cnt)


def brute(s_lo, s_hi, u_lo, u_hi, strict: bool = False) -> np.ndarray:
    d, n, m = _dims(s_lo, u_lo)
    a, pa = _f32(s_lo); b, pb = _f32(s_hi); c, pc = _f32(u_lo); e, pe = _f32(u_hi)
    keys = ctypes.POINTER(ctypes.c_uint64)()
    cnt = ctypes.c_uint64(0)
    rc = lib().oracle_brute(pa, pb, n, pc, pe, m, d, int(strict),
                            ctypes.byref(keys), ctypes.byref(cnt))
    return _take_keys(rc, keys, cnt)


def sbm_1d(s_lo, s_hi, u_lo, u_hi) -> np.ndarray:
    d, n, m = _dims(s_lo, u_lo)
    assert d == 1
    a, pa = _f32(s_lo); b, pb = _f32(s_hi); c, pc = _f32(u_lo); e, pe = _f32(u_hi)
    keys = ctypes.POINTER(ctypes.c_uint64)()
    cnt = ctypes.c_uint64(0)
    rc = lib().oracle_sbm_1d(pa, pb, n, pc, pe, m, ctypes.byref(keys), ctypes.byref(cnt))
    return _take_keys(rc, keys, cnt)


def itm_1d_visits(s_lo, s_hi, u_lo, u_hi):
    """Per-query node visits and hits of Algorithm 4, plus the tree height."""
    d, n, m = _dims(s_lo, u_lo)
    assert d == 1
    a, pa = _f32(s_lo); b, pb = _f32(s_hi); c, pc = _f32(u_lo); e, pe = _f32(u_hi)
    visits = np.zeros(m, dtype=np.uint64)
    hits = np.zeros(m, dtype=np.uint32)
    H = ctypes.c_uint32(0)
    rc = lib().oracle_itm_1d_visits(
        pa, pb, n, pc, pe, m,
        visits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        hits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(H))
    if rc != 0:
        raise OracleError(rc)
    return visits, hits, int(H.value)


def pst_1d(s_lo, s_hi, u_lo, u_hi):
    """Sorted keys from the priority search tree (d = 1), plus per-query
    nodes visited and hits."""
    d, n, m = _dims(s_lo, u_lo)
    assert d == 1
    a, pa = _f32(s_lo); b, pb = _f32(s_hi); c, pc = _f32(u_lo); e, pe = _f32(u_hi)
    keys = ctypes.POINTER(ctypes.c_uint64)()
    cnt = ctypes.c_uint64(0)
    visits = np.zeros(m, dtype=np.uint64)
    hits = np.zeros(m, dtype=np.uint32)
    rc = lib().oracle_pst_1d(pa, pb, n, pc, pe, m, ctypes.byref(keys), ctypes.byref(cnt),
                             visits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                             hits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return _take_keys(rc, keys, cnt), visits, hits


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def counts_per_update(keys: np.ndarray, m: int) -> np.ndarray:
    """Hits per update (segment lengths of the compressed column form of M)."""
    return np.bincount((keys >> np.uint64(32)).astype(np.int64), minlength=m).astype(np.uint32)


def expected_pairs_uniform(n: int, m: int, sides, L: float) -> float:
    """E[K] for lower corners uniform in [0, L)^d and common side s_k per axis.

    Per axis, two closed segments of length s with lower ends X, Y ~ U[0, L)
    meet iff |X - Y| <= s, probability 2 s / L - (s / L)^2 (s <= L); the axes
    are independent, and there are n * m pairs.
    """
    p = 1.0
    for s in sides:
        r = s / L
        p *= 2.0 * r - r * r
    return n * m * p
