"""ctypes binding of libddm.so (argument marshalling only).

Every computation happens in the library's HIP kernels.  If the library has
not been built this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_build", "libddm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "ddm.h")

DDM_OK = 0
DDM_E_INVALID_ARG = -1
DDM_E_INVALID_INPUT = -2
DDM_E_CAPACITY = -3
DDM_E_NOMEM = -4
DDM_E_DEVICE = -5
DDM_DYNAMIC_SUBSCRIPTIONS = 0
DDM_DYNAMIC_UPDATES = 1
DDM_NOALLOC_SCRATCH_MB = 64  # static scratch of ddm_match_noalloc (ddm.h)

TRAVERSE = {"auto": 0, "lane": 1, "tile": 2}
FEATURES = 18
PREDICTOR_PARAMS = 5441


class DDMError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        self.detail = detail
        msg = f"{where}: {strerror(code)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


class MatchOpts(ctypes.Structure):
    _fields_ = [("traversal", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 6)]


class BatchInstance(ctypes.Structure):
    _fields_ = [("sub_lo", ctypes.c_void_p), ("sub_hi", ctypes.c_void_p),
                ("upd_lo", ctypes.c_void_p), ("upd_hi", ctypes.c_void_p),
                ("n", ctypes.c_uint32), ("m", ctypes.c_uint32), ("d", ctypes.c_uint32),
                ("qpt", ctypes.c_uint32)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("qpt", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 5)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("host_pool", ctypes.c_uint64),
                ("workers", ctypes.c_uint32), ("tree_cache", ctypes.c_uint32),
                ("deliver_device", ctypes.c_uint32), ("batch_max", ctypes.c_uint32),
                ("batch_small", ctypes.c_uint32), ("compact", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 1)]


class Request(ctypes.Structure):
    _fields_ = [("sub_lo", ctypes.c_void_p), ("sub_hi", ctypes.c_void_p),
                ("upd_lo", ctypes.c_void_p), ("upd_hi", ctypes.c_void_p),
                ("n", ctypes.c_uint32), ("m", ctypes.c_uint32), ("d", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("tree_key", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("on_device", ctypes.c_uint32),
                ("count", ctypes.c_uint64), ("pairs", ctypes.c_void_p),
                ("t_arrival_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("slots", ctypes.c_uint64),
                ("overflowed", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("sub_ids", ctypes.c_void_p), ("upd_offsets", ctypes.c_void_p)]


class ServerCounters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("submitted", "completed", "queued", "in_flight", "hbm_used", "hbm_peak",
                 "host_pool_used", "trees_resident", "requeued")]


_lib = None

vp = ctypes.c_void_p
u32 = ctypes.c_uint32
u64 = ctypes.c_uint64
i32 = ctypes.c_int


def _sig(L, name, restype, *argtypes):
    f = getattr(L, name)
    f.restype = restype
    f.argtypes = list(argtypes)


def lib():
    """The loaded libddm (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libddm.so is not built ({LIB_PATH}); run "
            "`python -m paper_1309_3458_amd.build_lib` (or __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname as the system one;
    # loading torch first makes libddm bind to that runtime, so that the
    # library and torch's tensors and streams share one HIP runtime.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    _sig(L, "ddm_build", i32, vp, vp, u32, u32, vp, P(vp))
    _sig(L, "ddm_match", i32, vp, vp, vp, u32, vp, u64, P(u64), vp)
    _sig(L, "ddm_match_ex", i32, vp, vp, vp, u32, vp, u64, P(u64), vp, P(MatchOpts))
    _sig(L, "ddm_match_begin", i32, vp, vp, vp, u32, P(u64), vp, P(MatchOpts), P(vp))
    _sig(L, "ddm_match_finish", i32, vp, vp, u64)
    _sig(L, "ddm_match_abort", None, vp)
    _sig(L, "ddm_count", i32, vp, vp, vp, u32, vp, P(u64), vp, P(MatchOpts))
    _sig(L, "ddm_match_scratch_bytes", i32, u32, u32, u32, u64, P(u64))
    _sig(L, "ddm_match_noalloc", i32, vp, vp, vp, u32, vp, u64, P(u64), vp)
    _sig(L, "ddm_match_brute", i32, vp, vp, u32, vp, vp, u32, u32, vp, u64, P(u64), vp)
    _sig(L, "ddm_match_sbm", i32, vp, vp, u32, vp, vp, u32, u32, vp, u64, P(u64), vp)
    _sig(L, "ddm_match_sets", i32, vp, vp, u32, vp, vp, u32, u32, i32, vp, u64, P(u64),
         P(ctypes.c_int), vp)
    _sig(L, "ddm_tree_check", i32, vp)
    _sig(L, "ddm_tree_prepare_learned", i32, vp, vp)
    _sig(L, "ddm_dynamic_create", i32, vp, vp, u32, vp, vp, u32, u32, vp, P(vp))
    _sig(L, "ddm_dynamic_move", i32, vp, u32, vp, vp, vp, u32, vp, P(u64))
    _sig(L, "ddm_dynamic_result", i32, vp, P(vp), P(u64))
    _sig(L, "ddm_dynamic_free", None, vp)
    _sig(L, "ddm_tree_update", i32, vp, vp, vp, vp, u32, vp, P(i32))
    _sig(L, "ddm_tree_info", i32, vp, P(u32), P(u32), P(u32))
    _sig(L, "ddm_tree_export", i32, vp, u32, vp, vp, vp, vp)
    _sig(L, "ddm_tree_free", None, vp)
    _sig(L, "ddm_strerror", ctypes.c_char_p, i32)
    _sig(L, "ddm_last_error_detail", ctypes.c_char_p)
    _sig(L, "ddm_debug_alloc_cap", u64, u64)
    _sig(L, "ddm_prof_enable", None, i32)
    _sig(L, "ddm_prof_read", u64, ctypes.c_char_p, u64)
    _sig(L, "ddm_prof_focus", None, ctypes.c_char_p)
    f32p = ctypes.POINTER(ctypes.c_float)
    _sig(L, "ddm_predictor_create", i32, u64, P(vp))
    _sig(L, "ddm_predictor_free", None, vp)
    _sig(L, "ddm_predictor_get_params", i32, vp, vp, u32, f32p)
    _sig(L, "ddm_predictor_set_params", i32, vp, vp, u32, ctypes.c_float)
    _sig(L, "ddm_predictor_save", i32, vp, ctypes.c_char_p)
    _sig(L, "ddm_predictor_load", i32, ctypes.c_char_p, P(vp))
    _sig(L, "ddm_features", i32, vp, vp, vp, u32, vp, vp)
    _sig(L, "ddm_predictor_forward", i32, vp, vp, u32, vp, vp)
    _sig(L, "ddm_predictor_grad", i32, vp, vp, vp, u32, vp, vp, vp)
    _sig(L, "ddm_predictor_adam", i32, vp, vp, ctypes.c_float, vp)
    _sig(L, "ddm_predictor_train", i32, vp, vp, vp, u32, u32, u32, ctypes.c_float, vp, vp)
    _sig(L, "ddm_match_learned_begin", i32, vp, vp, vp, u32, vp, u64, P(u64), vp,
         P(MatchOpts), P(vp))
    _sig(L, "ddm_pending_info", i32, vp, P(u64), P(u64), P(u32))
    _sig(L, "ddm_batch_create", i32, P(BatchInstance), u32, vp, u64, P(BatchOpts), P(vp))
    _sig(L, "ddm_batch_run", i32, vp, vp)
    _sig(L, "ddm_batch_result", i32, vp, P(u64), vp)
    _sig(L, "ddm_batch_free", None, vp)
    _sig(L, "ddm_batch_count", i32, vp, vp, P(u64), vp)
    _sig(L, "ddm_batch_fill", i32, vp, vp, u64, vp)
    _sig(L, "ddm_server_create", i32, P(ServerOpts), vp, P(vp))
    _sig(L, "ddm_server_submit", i32, vp, P(Request), ctypes.c_int64, vp, P(u64))
    _sig(L, "ddm_server_wait_any", u32, vp, u32, vp, u32)
    _sig(L, "ddm_server_result", i32, vp, u64, P(Result))
    _sig(L, "ddm_server_release", i32, vp, u64)
    _sig(L, "ddm_server_stats", i32, vp, P(ServerCounters))
    _sig(L, "ddm_server_destroy", None, vp)
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().ddm_strerror(code).decode()
    except Exception:  # pragma: no cover - only when the library is missing
        return f"status {code}"


def check(code: int, where: str):
    if code != DDM_OK:
        raise DDMError(code, where, lib().ddm_last_error_detail().decode())


def header_functions() -> list[str]:
    """Names of every function the public header declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ddm_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def opts(traversal: str = "auto", block: int = 0) -> MatchOpts:
    o = MatchOpts()
    o.traversal = TRAVERSE[traversal]
    o.block = block
    return o
