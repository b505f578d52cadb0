"""ddm_match_noalloc (scratch in a static device array, no allocation)
through the C ABI: two calls in a row, the second smaller, each byte-identical
to ddm_match on the same inputs (and, for the small one, to the CPU oracle);
an update count beyond the static scratch and a too-small capacity fail
cleanly without writing any pair."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1309_3458_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(entry, tree, u_lo, u_hi, m, out, cap):
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    K = ctypes.c_uint64()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(N.lib(), entry)(tree, _ptr(u_lo), _ptr(u_hi), m,
                                 _ptr(out) if out is not None else None, cap, ctypes.byref(K), s)
    torch.cuda.synchronize()
    return rc, int(K.value)


def _build(inst):
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    s_lo, s_hi = dev(inst.s_lo), dev(inst.s_hi)
    h = ctypes.c_void_p()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert N.lib().ddm_build(_ptr(s_lo), _ptr(s_hi), inst.n, inst.d, s, ctypes.byref(h)) == 0
    return h, (s_lo, s_hi)


def _both(inst):
    """(noalloc keys, ddm_match keys) for one instance."""
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    h, keep = _build(inst)
    u_lo, u_hi = dev(inst.u_lo), dev(inst.u_hi)
    rc, K = _call("ddm_match", h, u_lo, u_hi, inst.m, None, 0)
    assert rc in (N.DDM_OK, N.DDM_E_CAPACITY)
    ref = torch.full((max(K, 1),), -1, dtype=torch.int64, device="cuda")
    rc, K1 = _call("ddm_match", h, u_lo, u_hi, inst.m, ref, ref.numel())
    assert rc == N.DDM_OK and K1 == K
    # the no-allocation buffer starts as garbage, so that an unwritten slot
    # cannot pass for a written one
    out = torch.full((max(K, 1),), -7, dtype=torch.int64, device="cuda")
    rc, K2 = _call("ddm_match_noalloc", h, u_lo, u_hi, inst.m, out, out.numel())
    assert rc == N.DDM_OK, N.lib().ddm_last_error_detail()
    assert K2 == K
    got = out[:K].cpu().numpy().view(np.uint64)
    want = ref[:K].cpu().numpy().view(np.uint64)
    N.lib().ddm_tree_free(h)
    del keep
    return got, want


def test_noalloc_two_calls_equal_ddm_match():
    big = W.uniform_instance(501, 400_000, 600_000, 2, W.side_for_alpha(1.0, 1_000_000, 2))
    got, want = _both(big)
    assert got.size > 100_000 and np.array_equal(got, want)
    small = W.uniform_instance(502, 30_000, 7_001, 3, W.side_for_alpha(5.0, 37_001, 3))
    got, want = _both(small)
    assert np.array_equal(got, want)
    assert np.array_equal(got, oracle.itm(small.s_lo, small.s_hi, small.u_lo, small.u_hi,
                                          threads=8))
    tiny = W.tiny_adversarial(503, 300, 129, 1)
    got, want = _both(tiny)
    assert np.array_equal(got, want)
    assert np.array_equal(got, oracle.itm(tiny.s_lo, tiny.s_hi, tiny.u_lo, tiny.u_hi))


def test_noalloc_limits_and_capacity():
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    inst = W.uniform_instance(504, 20_000, 5_000, 2, 5000.0)
    h, keep = _build(inst)
    u_lo, u_hi = dev(inst.u_lo), dev(inst.u_hi)
    rc, K = _call("ddm_match_noalloc", h, u_lo, u_hi, inst.m, None, 0)
    assert rc == N.DDM_E_CAPACITY and K > 0
    out = torch.full((K - 1,), -7, dtype=torch.int64, device="cuda")
    rc, K2 = _call("ddm_match_noalloc", h, u_lo, u_hi, inst.m, out, out.numel())
    assert rc == N.DDM_E_CAPACITY and K2 == K
    assert bool((out == -7).all())
    # more updates than the static scratch holds: refused before any kernel
    # runs (the buffers still hold m_big valid updates)
    b = ctypes.c_uint64()
    m_big = 2_000_000
    assert N.lib().ddm_match_scratch_bytes(m_big, 2, 0, 0, ctypes.byref(b)) == 0
    assert b.value > (N.DDM_NOALLOC_SCRATCH_MB << 20)
    big_lo = torch.zeros((2, m_big), dtype=torch.float32, device="cuda")
    big_hi = torch.ones((2, m_big), dtype=torch.float32, device="cuda")
    rc, _ = _call("ddm_match_noalloc", h, big_lo, big_hi, m_big, out, out.numel())
    assert rc == N.DDM_E_INVALID_ARG
    assert "static" in N.lib().ddm_last_error_detail().decode() or \
        "scratch" in N.lib().ddm_last_error_detail().decode()
    assert bool((out == -7).all())
    N.lib().ddm_tree_free(h)
    del keep
