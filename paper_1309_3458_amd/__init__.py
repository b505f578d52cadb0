"""Interval Tree Matching for DDM on MI355X (gfx950).

Python face of libddm.  Tensors are torch CUDA tensors used as device memory;
all work runs in the library's HIP kernels on the current torch stream.

    tree = build(s_lo, s_hi)          # float32 [d, n] each, on the GPU
    keys = match(tree, u_lo, u_hi)    # int64 [K]: (update << 32) | subscription
"""
from __future__ import annotations

import ctypes
import json
import os

from ._native import (DDMError, DDM_E_CAPACITY, DDM_E_INVALID_INPUT, FEATURES, PREDICTOR_PARAMS,
                      TRAVERSE, check, header_functions, lib, opts as _opts)

__all__ = ["build", "match", "count", "Tree", "DDMError", "prof_enable", "prof_read",
           "TRAVERSE", "header_functions", "Predictor", "features", "match_learned", "Batch",
           "Server", "Dynamic", "match_brute", "match_sbm",
           "match_sets", "SWAP_AUTO", "SWAP_NEVER", "SWAP_ALWAYS"]


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _coords(lo, hi, what):
    torch = _torch()
    if lo.dtype != torch.float32 or hi.dtype != torch.float32:
        raise TypeError(f"{what}: coordinates must be float32")
    if lo.dim() != 2 or lo.shape != hi.shape:
        raise ValueError(f"{what}: expected lo, hi of equal shape [d, count]")
    if not lo.is_cuda or not hi.is_cuda:
        raise ValueError(f"{what}: tensors must be on the GPU")
    return lo.contiguous(), hi.contiguous()


class Tree:
    """Handle of per-dimension interval trees built on the device."""

    def __init__(self, handle: ctypes.c_void_p, n: int, d: int, keep):
        self._h = handle
        self.n = n
        self.d = d
        self._keep = keep  # inputs stay alive until the build has run

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("tree already freed")
        return self._h

    def check(self):
        check(lib().ddm_tree_check(self.handle), "ddm_tree_check")

    def prepare_learned(self, stream=None):
        """Enqueue the statistics the learned path's features read now,
        instead of in the first learned match (d <= 3, n > 0)."""
        check(lib().ddm_tree_prepare_learned(self.handle, _stream_handle(stream)),
              "ddm_tree_prepare_learned")

    def info(self):
        n, d, h = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        check(lib().ddm_tree_info(self.handle, ctypes.byref(n), ctypes.byref(d),
                                  ctypes.byref(h)), "ddm_tree_info")
        return n.value, d.value, h.value

    def export(self, k: int):
        """(lo, hi, ids, maxhi) numpy arrays of dimension k's tree (in order)."""
        import numpy as np
        n, d, H = self.info()
        lo = np.zeros(n, np.float32)
        hi = np.zeros(n, np.float32)
        ids = np.zeros(n, np.uint32)
        mx = np.zeros((1 << H) - 1 if H else 0, np.float32)
        check(lib().ddm_tree_export(self.handle, k, lo.ctypes.data, hi.ctypes.data,
                                    ids.ctypes.data, mx.ctypes.data), "ddm_tree_export")
        return lo, hi, ids, mx

    def update(self, ids, new_lo, new_hi, stream=None) -> bool:
        """Move subscriptions `ids` (int32/uint32 GPU tensor) to new extents
        ([d, count] float32 GPU tensors); True if the tree was rebuilt, False
        if it was refitted in place."""
        torch = _torch()
        new_lo, new_hi = _coords(new_lo, new_hi, "Tree.update")
        if ids.dtype not in (torch.int32, torch.uint32) or not ids.is_cuda:
            raise TypeError("Tree.update: ids must be an int32 GPU tensor")
        ids = ids.contiguous()
        if new_lo.shape != (self.d, ids.numel()):
            raise ValueError("Tree.update: new extents must be [d, len(ids)]")
        rb = ctypes.c_int()
        check(lib().ddm_tree_update(self.handle, _ptr(ids), _ptr(new_lo), _ptr(new_hi),
                                    ids.numel(), _stream_handle(stream), ctypes.byref(rb)),
              "ddm_tree_update")
        return bool(rb.value)

    def free(self):
        if self._h is not None:
            lib().ddm_tree_free(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build(s_lo, s_hi, stream=None) -> Tree:
    """Interval trees over subscriptions s_lo, s_hi (float32 [d, n] on the GPU)."""
    s_lo, s_hi = _coords(s_lo, s_hi, "build")
    d, n = int(s_lo.shape[0]), int(s_lo.shape[1])
    h = ctypes.c_void_p()
    check(lib().ddm_build(ctypes.c_void_p(s_lo.data_ptr()), ctypes.c_void_p(s_hi.data_ptr()),
                          n, d, _stream_handle(stream), ctypes.byref(h)), "ddm_build")
    return Tree(h, n, d, (s_lo, s_hi))


def match(tree: Tree, u_lo, u_hi, traversal: str = "auto", block: int = 0, stream=None,
          out=None):
    """Sorted int64 keys (update << 32) | subscription of all intersecting pairs.

    With ``out`` (int64 CUDA tensor) the keys are written into its first K
    slots and a view of them is returned; otherwise a tensor of exactly K
    elements is allocated on the current stream.
    """
    torch = _torch()
    u_lo, u_hi = _coords(u_lo, u_hi, "match")
    if u_lo.shape[0] != tree.d:
        raise ValueError("match: update dimension differs from the tree's")
    m = int(u_lo.shape[1])
    o = _opts(traversal, block)
    K = ctypes.c_uint64()
    pend = ctypes.c_void_p()
    sh = _stream_handle(stream)
    check(lib().ddm_match_begin(tree.handle, ctypes.c_void_p(u_lo.data_ptr()),
                                ctypes.c_void_p(u_hi.data_ptr()), m, ctypes.byref(K), sh,
                                ctypes.byref(o), ctypes.byref(pend)), "ddm_match_begin")
    k = int(K.value)
    if out is None:
        dev = u_lo.device
        out = torch.empty(k, dtype=torch.int64, device=dev)
    elif out.dtype != torch.int64 or not out.is_cuda:
        lib().ddm_match_abort(pend)
        raise TypeError("match: out must be an int64 CUDA tensor")
    if out.numel() < k:
        lib().ddm_match_abort(pend)
        raise DDMError(DDM_E_CAPACITY, "match", f"K={k} > capacity {out.numel()}")
    ptr = ctypes.c_void_p(out.data_ptr()) if out.numel() else ctypes.c_void_p()
    check(lib().ddm_match_finish(pend, ptr, out.numel()), "ddm_match_finish")
    return out[:k]


def match_into(tree: Tree, u_lo, u_hi, out, traversal: str = "auto", block: int = 0,
               stream=None) -> int:
    """One-call form (ddm_match_ex): writes into ``out`` and returns K.

    Raises DDMError(DDM_E_CAPACITY) with ``.detail`` holding K if out is too
    small.
    """
    u_lo, u_hi = _coords(u_lo, u_hi, "match_into")
    m = int(u_lo.shape[1])
    o = _opts(traversal, block)
    K = ctypes.c_uint64()
    ptr = ctypes.c_void_p(out.data_ptr()) if out.numel() else ctypes.c_void_p()
    rc = lib().ddm_match_ex(tree.handle, ctypes.c_void_p(u_lo.data_ptr()),
                            ctypes.c_void_p(u_hi.data_ptr()), m, ptr, out.numel(),
                            ctypes.byref(K), _stream_handle(stream), ctypes.byref(o))
    if rc == DDM_E_CAPACITY:
        raise DDMError(rc, "ddm_match_ex", str(int(K.value)))
    check(rc, "ddm_match_ex")
    return int(K.value)


def count(tree: Tree, u_lo, u_hi, traversal: str = "auto", block: int = 0, stream=None):
    """(counts int32 [m], K): subscriptions met by each update."""
    torch = _torch()
    u_lo, u_hi = _coords(u_lo, u_hi, "count")
    m = int(u_lo.shape[1])
    counts = torch.empty(m, dtype=torch.int32, device=u_lo.device)
    o = _opts(traversal, block)
    K = ctypes.c_uint64()
    check(lib().ddm_count(tree.handle, ctypes.c_void_p(u_lo.data_ptr()),
                          ctypes.c_void_p(u_hi.data_ptr()), m,
                          ctypes.c_void_p(counts.data_ptr()) if m else ctypes.c_void_p(),
                          ctypes.byref(K), _stream_handle(stream), ctypes.byref(o)),
          "ddm_count")
    return counts, int(K.value)


def _match_pairwise(entry: str, s_lo, s_hi, u_lo, u_hi, stream, out):
    torch = _torch()
    s_lo, s_hi = _coords(s_lo, s_hi, f"{entry} subscriptions")
    u_lo, u_hi = _coords(u_lo, u_hi, f"{entry} updates")
    if s_lo.shape[0] != u_lo.shape[0]:
        raise ValueError(f"{entry}: subscriptions and updates differ in d")
    n, m, d = int(s_lo.shape[1]), int(u_lo.shape[1]), int(s_lo.shape[0])
    fn = getattr(lib(), entry)
    K = ctypes.c_uint64()
    h = _stream_handle(stream)
    cap = out.numel() if out is not None else 0
    code = fn(_ptr(s_lo), _ptr(s_hi), n, _ptr(u_lo), _ptr(u_hi), m, d,
              _ptr(out) if out is not None else None, cap, ctypes.byref(K), h)
    if out is None and code == DDM_E_CAPACITY:
        out = torch.empty(int(K.value), dtype=torch.int64, device=u_lo.device)
        code = fn(_ptr(s_lo), _ptr(s_hi), n, _ptr(u_lo), _ptr(u_hi), m, d,
                  _ptr(out), out.numel(), ctypes.byref(K), h)
    check(code, entry)
    if out is None:
        out = torch.empty(0, dtype=torch.int64, device=u_lo.device)
    return out[:int(K.value)]


def match_brute(s_lo, s_hi, u_lo, u_hi, stream=None, out=None):
    """Brute-force matching on the GPU (the paper's baseline); same keys as
    build() + match()."""
    return _match_pairwise("ddm_match_brute", s_lo, s_hi, u_lo, u_hi, stream, out)


def match_sbm(s_lo, s_hi, u_lo, u_hi, stream=None, out=None):
    """Sort-based matching on the GPU (the paper's sweep-line comparison
    system); same keys as build() + match()."""
    return _match_pairwise("ddm_match_sbm", s_lo, s_hi, u_lo, u_hi, stream, out)


SWAP_AUTO, SWAP_NEVER, SWAP_ALWAYS = 0, 1, 2


def match_sets(s_lo, s_hi, u_lo, u_hi, swap=SWAP_AUTO, stream=None, out=None,
               return_swapped=False):
    """build() + match() for two sets given together, optionally with the
    tree on the smaller set (roles of subscriptions and updates swapped when
    n > m and d >= 3 under SWAP_AUTO, always under SWAP_ALWAYS); the keys
    are the same as build(s) + match(u)."""
    torch = _torch()
    s_lo, s_hi = _coords(s_lo, s_hi, "match_sets subscriptions")
    u_lo, u_hi = _coords(u_lo, u_hi, "match_sets updates")
    if s_lo.shape[0] != u_lo.shape[0]:
        raise ValueError("match_sets: subscriptions and updates differ in d")
    n, m, d = int(s_lo.shape[1]), int(u_lo.shape[1]), int(s_lo.shape[0])
    K = ctypes.c_uint64()
    sw = ctypes.c_int(0)
    h = _stream_handle(stream)

    def call(buf):
        return lib().ddm_match_sets(_ptr(s_lo), _ptr(s_hi), n, _ptr(u_lo), _ptr(u_hi), m, d,
                                    int(swap), _ptr(buf) if buf is not None else None,
                                    buf.numel() if buf is not None else 0, ctypes.byref(K),
                                    ctypes.byref(sw), h)

    code = call(out)
    if out is None and code == DDM_E_CAPACITY:
        out = torch.empty(int(K.value), dtype=torch.int64, device=u_lo.device)
        code = call(out)
    check(code, "ddm_match_sets")
    if out is None:
        out = torch.empty(0, dtype=torch.int64, device=u_lo.device)
    res = out[:int(K.value)]
    return (res, bool(sw.value)) if return_swapped else res


def prof_enable(on: bool = True, only: str | None = None):
    """Record HIP events around kernel launches (optionally one kernel only)."""
    lib().ddm_prof_focus(only.encode() if only else None)
    lib().ddm_prof_enable(1 if on else 0)


def prof_read() -> dict:
    """{kernel: (total_ms, launches)} since the last read (waits for events)."""
    buf = ctypes.create_string_buffer(1 << 16)
    need = lib().ddm_prof_read(buf, len(buf))
    if need >= len(buf):
        raise RuntimeError("kernel timing report truncated")
    return {k: tuple(v) for k, v in json.loads(buf.value.decode()).items()}


# ---------------------------------------------------------------------------
# learned output sizing
# ---------------------------------------------------------------------------
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p()


class Predictor:
    """Hit-count predictor (MLP 18 -> 64 -> 64 -> 1, FP32) living on the GPU."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        check(lib().ddm_predictor_create(seed, ctypes.byref(h)), "ddm_predictor_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self):
        import numpy as np
        a = np.zeros(PREDICTOR_PARAMS, np.float32)
        d = ctypes.c_float()
        check(lib().ddm_predictor_get_params(self._h, a.ctypes.data, PREDICTOR_PARAMS,
                                             ctypes.byref(d)), "ddm_predictor_get_params")
        return a, float(d.value)

    def set_params(self, params=None, delta: float | None = None):
        import numpy as np
        if delta is None:
            delta = self.params()[1]
        if params is None:
            check(lib().ddm_predictor_set_params(self._h, None, 0, float(delta)),
                  "ddm_predictor_set_params")
            return
        a = np.ascontiguousarray(params, dtype=np.float32)
        assert a.size == PREDICTOR_PARAMS
        check(lib().ddm_predictor_set_params(self._h, a.ctypes.data, PREDICTOR_PARAMS,
                                             float(delta)), "ddm_predictor_set_params")

    @property
    def delta(self) -> float:
        return self.params()[1]

    def forward(self, X, stream=None):
        torch = _torch()
        X = X.contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        check(lib().ddm_predictor_forward(self._h, _ptr(X), X.shape[0], _ptr(y),
                                          _stream_handle(stream)), "ddm_predictor_forward")
        return y

    def grad(self, X, Y, stream=None):
        torch = _torch()
        X, Y = X.contiguous(), Y.contiguous()
        g = torch.empty(PREDICTOR_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        check(lib().ddm_predictor_grad(self._h, _ptr(X), _ptr(Y), X.shape[0], _ptr(g), _ptr(loss),
                                       _stream_handle(stream)), "ddm_predictor_grad")
        return g, loss

    def adam(self, grad, lr: float, stream=None):
        check(lib().ddm_predictor_adam(self._h, _ptr(grad), float(lr), _stream_handle(stream)),
              "ddm_predictor_adam")

    def train(self, X, Y, batch: int = 4096, epochs: int = 10, lr: float = 1e-3, stream=None):
        import numpy as np
        X, Y = X.contiguous(), Y.contiguous()
        losses = np.zeros(epochs, np.float32)
        check(lib().ddm_predictor_train(self._h, _ptr(X), _ptr(Y), X.shape[0], batch, epochs,
                                        float(lr), _stream_handle(stream), losses.ctypes.data),
              "ddm_predictor_train")
        return losses

    def save(self, path: str):
        """Parameters and delta to a predictor file (ddm_predictor_save)."""
        check(lib().ddm_predictor_save(self.handle, os.fsencode(path)), "ddm_predictor_save")

    @classmethod
    def load(cls, path: str):
        """A new predictor from a file written by save() (ddm_predictor_load)."""
        h = ctypes.c_void_p()
        check(lib().ddm_predictor_load(os.fsencode(path), ctypes.byref(h)), "ddm_predictor_load")
        p = cls.__new__(cls)
        p._h = h
        return p

    def free(self):
        if self._h is not None:
            lib().ddm_predictor_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def features(tree: Tree, u_lo, u_hi, stream=None):
    """float32 [m, 18] features of the updates against the tree (d <= 3)."""
    torch = _torch()
    u_lo, u_hi = _coords(u_lo, u_hi, "features")
    m = int(u_lo.shape[1])
    X = torch.empty((m, FEATURES), dtype=torch.float32, device=u_lo.device)
    check(lib().ddm_features(tree.handle, _ptr(u_lo), _ptr(u_hi), m, _ptr(X),
                             _stream_handle(stream)), "ddm_features")
    return X


def match_learned(tree: Tree, u_lo, u_hi, predictor: Predictor, slot_budget: int = 0,
                  traversal: str = "auto", block: int = 0, stream=None, out=None,
                  info: dict | None = None):
    """Single-pass match sized by the predictor; same keys as match()."""
    torch = _torch()
    u_lo, u_hi = _coords(u_lo, u_hi, "match_learned")
    m = int(u_lo.shape[1])
    o = _opts(traversal, block)
    K = ctypes.c_uint64()
    pend = ctypes.c_void_p()
    check(lib().ddm_match_learned_begin(tree.handle, _ptr(u_lo), _ptr(u_hi), m, predictor.handle,
                                        int(slot_budget), ctypes.byref(K),
                                        _stream_handle(stream), ctypes.byref(o),
                                        ctypes.byref(pend)), "ddm_match_learned_begin")
    if info is not None and pend:
        sl, bu, ov = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
        lib().ddm_pending_info(pend, ctypes.byref(sl), ctypes.byref(bu), ctypes.byref(ov))
        info.update(slots=int(sl.value), budget=int(bu.value), overflowed=int(ov.value))
    k = int(K.value)
    if out is None:
        out = torch.empty(k, dtype=torch.int64, device=u_lo.device)
    if out.numel() < k:
        lib().ddm_match_abort(pend)
        raise DDMError(DDM_E_CAPACITY, "match_learned", f"K={k} > capacity {out.numel()}")
    check(lib().ddm_match_finish(pend, _ptr(out), out.numel()), "ddm_match_finish")
    return out[:k]


class Dynamic:
    """Both extent sets, a tree over each and the current result kept on the
    device (ddm_dynamic_*): move(set, ids, new_lo, new_hi) moves extents of
    one set and recomputes only their pairs; pairs() is the current sorted
    result (int64 keys (update << 32) | subscription)."""

    SUBSCRIPTIONS = 0
    UPDATES = 1

    def __init__(self, s_lo, s_hi, u_lo, u_hi, stream=None):
        s_lo, s_hi = _coords(s_lo, s_hi, "Dynamic subscriptions")
        u_lo, u_hi = _coords(u_lo, u_hi, "Dynamic updates")
        if s_lo.shape[0] != u_lo.shape[0]:
            raise ValueError("Dynamic: subscriptions and updates differ in d")
        self.d, self.n, self.m = int(s_lo.shape[0]), int(s_lo.shape[1]), int(u_lo.shape[1])
        h = ctypes.c_void_p()
        check(lib().ddm_dynamic_create(_ptr(s_lo), _ptr(s_hi), self.n, _ptr(u_lo), _ptr(u_hi),
                                       self.m, self.d, _stream_handle(stream), ctypes.byref(h)),
              "ddm_dynamic_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("dynamic matcher already freed")
        return self._h

    def move(self, which: int, ids, new_lo, new_hi, stream=None) -> int:
        """Moves extents ids (int32/uint32 GPU tensor, distinct) of set
        `which` (SUBSCRIPTIONS or UPDATES) to new_lo/new_hi (float32 [d, c]
        GPU tensors); returns the new pair count."""
        torch = _torch()
        new_lo, new_hi = _coords(new_lo, new_hi, "Dynamic.move")
        if ids.dtype not in (torch.int32,) or not ids.is_cuda:
            raise TypeError("Dynamic.move: ids must be an int32 CUDA tensor")
        ids = ids.contiguous()
        K = ctypes.c_uint64()
        check(lib().ddm_dynamic_move(self.handle, int(which), _ptr(ids) if ids.numel() else None,
                                     _ptr(new_lo), _ptr(new_hi), int(ids.numel()),
                                     _stream_handle(stream), ctypes.byref(K)),
              "ddm_dynamic_move")
        return int(K.value)

    def pairs(self):
        """A copy of the current result (int64 CUDA tensor)."""
        torch = _torch()
        p, K = ctypes.c_void_p(), ctypes.c_uint64()
        check(lib().ddm_dynamic_result(self.handle, ctypes.byref(p), ctypes.byref(K)),
              "ddm_dynamic_result")
        k = int(K.value)
        if k == 0:
            return torch.zeros(0, dtype=torch.int64, device="cuda")

        class _Dev:  # a view of the library's device buffer
            __cuda_array_interface__ = {"shape": (k,), "typestr": "<i8",
                                        "data": (int(p.value), False), "version": 2}

        return torch.as_tensor(_Dev(), device="cuda").clone()

    def free(self):
        if self._h is not None:
            lib().ddm_dynamic_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Many independent instances matched by one fixed kernel sequence.

    instances: list of (s_lo, s_hi, u_lo, u_hi) float32 GPU tensors, [d, n]
    and [d, m].  The output buffer (int64, `capacity` keys) is allocated
    here; after run() + result(), pairs(i) is instance i's sorted keys (the
    bytes match() returns for that instance alone).  qpts optionally gives
    each instance's work-item size (16, 32 or 64; see tune.py), qpt and
    waves_per_cu the batch defaults.  The coordinate tensors
    may be overwritten in place between runs (same shapes).
    """

    def __init__(self, instances, capacity: int, qpt: int = 64, waves_per_cu: int = 0,
                 use_graph: bool = True, out=None, qpts=None):
        from ._native import BatchInstance, BatchOpts
        torch = _torch()
        keep = []
        arr = (BatchInstance * len(instances))()
        for i, (s_lo, s_hi, u_lo, u_hi) in enumerate(instances):
            s_lo, s_hi = _coords(s_lo, s_hi, "Batch subscriptions")
            u_lo, u_hi = _coords(u_lo, u_hi, "Batch updates")
            if s_lo.shape[0] != u_lo.shape[0]:
                raise ValueError("Batch: subscriptions and updates differ in d")
            keep += [s_lo, s_hi, u_lo, u_hi]
            arr[i].sub_lo, arr[i].sub_hi = _ptr(s_lo), _ptr(s_hi)
            arr[i].upd_lo, arr[i].upd_hi = _ptr(u_lo), _ptr(u_hi)
            arr[i].n, arr[i].m, arr[i].d = int(s_lo.shape[1]), int(u_lo.shape[1]), int(s_lo.shape[0])
            arr[i].qpt = int(qpts[i]) if qpts is not None else 0
        if out is None:
            dev = keep[0].device if keep else "cuda"
            out = torch.empty(max(1, int(capacity)), dtype=torch.int64, device=dev)
        self.out = out
        self.count = len(instances)
        self._keep = keep
        o = BatchOpts()
        o.qpt, o.waves_per_cu, o.use_graph = int(qpt), int(waves_per_cu), int(bool(use_graph))
        h = ctypes.c_void_p()
        check(lib().ddm_batch_create(arr, len(instances), _ptr(out), int(capacity),
                                     ctypes.byref(o), ctypes.byref(h)), "ddm_batch_create")
        self._h = h
        self._ranges = None

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("batch already freed")
        return self._h

    def run(self, stream=None):
        self._ranges = None
        check(lib().ddm_batch_run(self.handle, _stream_handle(stream)), "ddm_batch_run")

    def result(self):
        """(total pairs, host list of count + 1 offsets); raises on overflow."""
        import numpy as np
        tot = ctypes.c_uint64()
        rg = np.zeros(self.count + 1, dtype=np.uint64)
        code = lib().ddm_batch_result(self.handle, ctypes.byref(tot),
                                      rg.ctypes.data_as(ctypes.c_void_p))
        self.total = int(tot.value)
        self._ranges = rg
        check(code, "ddm_batch_result")
        return self.total, rg

    def count_pairs(self, stream=None):
        """Two-step form (batches without a graph): the total and the
        instance offsets, before any output exists."""
        import numpy as np
        tot = ctypes.c_uint64()
        rg = np.zeros(self.count + 1, dtype=np.uint64)
        check(lib().ddm_batch_count(self.handle, _stream_handle(stream), ctypes.byref(tot),
                                    rg.ctypes.data_as(ctypes.c_void_p)), "ddm_batch_count")
        self.total, self._ranges = int(tot.value), rg
        return self.total, rg

    def fill(self, out, stream=None):
        """Second step: the pairs into `out` (int64 GPU tensor)."""
        check(lib().ddm_batch_fill(self.handle, _ptr(out), out.numel(), _stream_handle(stream)),
              "ddm_batch_fill")
        self.out = out

    def pairs(self, i: int):
        if self._ranges is None:
            self.result()
        a, b = int(self._ranges[i]), int(self._ranges[i + 1])
        return self.out[a:b]

    def free(self):
        if self._h is not None:
            lib().ddm_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Concurrent matching of requests that arrive at any time (ddm_server_*).

    submit() queues (s_lo, s_hi, u_lo, u_hi) GPU tensors and returns a
    ticket; the tensors are kept alive until the ticket is released.
    wait_any() blocks (releasing the GIL) until requests complete;
    result(ticket) returns a dict with the status, timestamps and, when
    `copy` is set, a numpy copy of the result: the sorted keys (uint64,
    "pairs") or, for a compact server, the subscription ids ("sub_ids") and
    the update offsets ("upd_offsets").
    """

    def __init__(self, predictor: Predictor | None = None, hbm_budget: int = 0,
                 host_pool: int = 0, workers: int = 8, tree_cache: int = 0,
                 deliver_device: bool = False, batch_max: int = 0, batch_small: int = 0,
                 compact: bool = False):
        from ._native import ServerOpts
        o = ServerOpts()
        o.hbm_budget, o.host_pool = int(hbm_budget), int(host_pool)
        o.workers, o.tree_cache, o.deliver_device = int(workers), int(tree_cache), \
            int(bool(deliver_device))
        o.batch_max, o.batch_small, o.compact = int(batch_max), int(batch_small), \
            int(bool(compact))
        h = ctypes.c_void_p()
        check(lib().ddm_server_create(ctypes.byref(o),
                                      predictor.handle if predictor is not None else None,
                                      ctypes.byref(h)), "ddm_server_create")
        self._h = h
        self._pred = predictor
        self._keep = {}
        self.deliver_device = bool(deliver_device)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("server already destroyed")
        return self._h

    def submit(self, s_lo, s_hi, u_lo, u_hi, tree_key: int = 0, arrival_ns: int = 0,
               stream=None) -> int:
        from ._native import Request
        u_lo, u_hi = _coords(u_lo, u_hi, "Server updates")
        r = Request()
        keep = [u_lo, u_hi]
        if s_lo is not None:
            s_lo, s_hi = _coords(s_lo, s_hi, "Server subscriptions")
            keep += [s_lo, s_hi]
            r.sub_lo, r.sub_hi, r.n = _ptr(s_lo), _ptr(s_hi), int(s_lo.shape[1])
        r.upd_lo, r.upd_hi = _ptr(u_lo), _ptr(u_hi)
        r.m, r.d, r.tree_key = int(u_lo.shape[1]), int(u_lo.shape[0]), int(tree_key)
        t = ctypes.c_uint64()
        check(lib().ddm_server_submit(self.handle, ctypes.byref(r), int(arrival_ns),
                                      _stream_handle(stream), ctypes.byref(t)),
              "ddm_server_submit")
        self._keep[int(t.value)] = keep
        return int(t.value)

    def wait_any(self, timeout_ms: int = 100, max_tickets: int = 1024) -> list[int]:
        buf = (ctypes.c_uint64 * max_tickets)()
        n = lib().ddm_server_wait_any(self.handle, int(timeout_ms), buf, max_tickets)
        return [int(buf[i]) for i in range(n)]

    def result(self, ticket: int, copy: bool = True) -> dict:
        import numpy as np
        from ._native import Result
        r = Result()
        check(lib().ddm_server_result(self.handle, int(ticket), ctypes.byref(r)),
              "ddm_server_result")
        d = {"status": int(r.status), "count": int(r.count), "t_arrival_ns": int(r.t_arrival_ns),
             "t_start_ns": int(r.t_start_ns), "t_done_ns": int(r.t_done_ns),
             "slots": int(r.slots), "overflowed": int(r.overflowed)}
        if r.status not in (0, 1):
            d["detail"] = lib().ddm_last_error_detail().decode()
        if copy and r.status == 0:
            if r.sub_ids is not None or r.upd_offsets is not None:
                # compact form (copied as the library delivers it): subscription
                # ids of every pair, and each update's first pair
                K, m = int(r.count), int(r.m)
                ids = np.frombuffer((ctypes.c_uint32 * K).from_address(int(r.sub_ids)),
                                    dtype=np.uint32).copy() if K else np.zeros(0, np.uint32)
                off = np.frombuffer((ctypes.c_uint64 * (m + 1)).from_address(int(r.upd_offsets)),
                                    dtype=np.uint64).copy()
                d["sub_ids"], d["upd_offsets"] = ids, off
            elif r.count == 0:
                d["pairs"] = np.zeros(0, dtype=np.uint64)
            elif r.on_device:
                torch = _torch()

                class _Dev:  # a view of the server's device buffer
                    __cuda_array_interface__ = {"shape": (int(r.count),), "typestr": "<i8",
                                                "data": (int(r.pairs), False), "version": 2}

                d["pairs"] = torch.as_tensor(_Dev(), device="cuda").cpu().numpy().view(np.uint64)
            else:
                buf = (ctypes.c_uint64 * int(r.count)).from_address(int(r.pairs))
                d["pairs"] = np.frombuffer(buf, dtype=np.uint64).copy()
        return d

    def release(self, ticket: int):
        check(lib().ddm_server_release(self.handle, int(ticket)), "ddm_server_release")
        self._keep.pop(int(ticket), None)

    def stats(self) -> dict:
        from ._native import ServerCounters
        c = ServerCounters()
        check(lib().ddm_server_stats(self.handle, ctypes.byref(c)), "ddm_server_stats")
        return {k: int(getattr(c, k)) for k, _ in ServerCounters._fields_}

    def close(self):
        if self._h is not None:
            lib().ddm_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
