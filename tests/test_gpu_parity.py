"""GPU path vs the CPU oracle, through the C ABI (libddm) on one GPU.

Integer results (pair keys, counts, tree ids) must be bit-exact.  Sizes span
several 64-update tiles, 4096-key sort tiles and a ragged tail; the 1M-region
2-D workload is checked at full size on sampled updates (the oracle computes
each sampled update's column of M) and through size-independent properties.
"""
import numpy as np
import pytest

import oracle
from paper_1309_3458_amd import workloads as W

pytestmark = pytest.mark.gpu

TRAVERSALS = ["tile", "lane"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_match(inst, traversal="auto", block=0):
    import paper_1309_3458_amd as P
    torch = _torch()
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    keys = P.match(t, dev(inst.u_lo), dev(inst.u_hi), traversal=traversal, block=block)
    torch.cuda.synchronize()
    out = keys.cpu().numpy().view(np.uint64)
    t.free()
    return out


def assert_keys_equal(got, want):
    assert got.shape == want.shape, (got.shape, want.shape)
    if got.size:
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"first mismatch at {bad[0]}: {got[bad[0]]:#x} vs {want[bad[0]]:#x}"


@pytest.mark.parametrize("traversal", TRAVERSALS)
def test_small_1d_full(traversal):
    inst = W.small_1d(0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert_keys_equal(gpu_match(inst, traversal), want)


@pytest.mark.parametrize("traversal", TRAVERSALS)
@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("n,m", [(1, 1), (63, 65), (64, 64), (65, 129), (700, 4097),
                                 (4097, 300)])
def test_adversarial_ties(traversal, d, n, m):
    inst = W.tiny_adversarial(n * 7 + m + d, n, m, d, grid=12)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert_keys_equal(gpu_match(inst, traversal), want)


@pytest.mark.parametrize("traversal", TRAVERSALS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_variable_lengths(traversal, d):
    inst = W.random_lengths(50 + d, 20011, 17003, d, L=5000.0, max_len=60.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert_keys_equal(gpu_match(inst, traversal), want)


@pytest.mark.parametrize("block", [64, 1024])
def test_lane_block_sizes(block):
    inst = W.random_lengths(77, 5000, 3001, 2, L=2000.0, max_len=40.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert_keys_equal(gpu_match(inst, "lane", block), want)


def test_long_segments():
    # few subscriptions, wide updates: segments of thousands of keys exercise
    # the LDS bitonic and bitmap segment sorts
    rng = np.random.default_rng(9)
    n, m = 30000, 300
    s_lo = rng.uniform(0, 1000, (2, n)).astype(np.float32)
    s_hi = (s_lo + np.float32(5)).astype(np.float32)
    u_lo = rng.uniform(0, 1000, (2, m)).astype(np.float32)
    w = rng.choice([10.0, 300.0, 900.0], size=(1, m)).astype(np.float32)
    u_hi = (u_lo + w).astype(np.float32)
    inst = W.Instance(s_lo, s_hi, u_lo, u_hi)
    want = oracle.itm(s_lo, s_hi, u_lo, u_hi, threads=8)
    cnt = oracle.counts_per_update(want, m)
    assert cnt.max() > 4096 and ((cnt > 16) & (cnt <= 4096)).any()
    for tr in TRAVERSALS:
        assert_keys_equal(gpu_match(inst, tr), want)


def test_long_segment_chunk_boundaries():
    """Segments of more than 8192 keys are read back from the bitmap sort's
    marks in staged chunks; with 10^5 ids a chunk holds 2 * ceil(w4 / 4) +
    2048 = 2440 positions (w4 = 782 uint4 entries).  Unit points in shuffled
    id order and updates covering exactly L consecutive points give segments
    of exactly L keys: L at and around the register window's rounds of
    1024 ids and its end (8192), at multiples of the chunk and the whole
    set; plain (tile and lane forms) and the learned single pass."""
    import paper_1309_3458_amd as P
    torch = _torch()
    rng = np.random.default_rng(23)
    n, chunk = 100000, 2440
    pos = rng.permutation(n).astype(np.float32)
    s_lo = pos[None, :].copy()
    s_hi = pos[None, :].copy()
    # the register window's rounds of 1024 ids: whole, ending exactly, one past
    lens = [2049, 3071, 3072, 3073, 4096, 5000, 7168,
            8191, 8192, 8193, 4 * chunk - 1, 4 * chunk, 4 * chunk + 1, 5 * chunk,
            8 * chunk + 1, 30000, n]
    starts = [int(rng.integers(0, n - L + 1)) for L in lens]
    u_lo = np.asarray([starts], np.float32)
    u_hi = np.asarray([[a + L - 1 for a, L in zip(starts, lens)]], np.float32)
    inst = W.Instance(s_lo, s_hi, u_lo, u_hi)
    want = oracle.itm(s_lo, s_hi, u_lo, u_hi, threads=8)
    assert np.array_equal(oracle.counts_per_update(want, len(lens)), lens)
    for tr in TRAVERSALS:
        assert_keys_equal(gpu_match(inst, tr), want)
    t = P.build(dev(s_lo), dev(s_hi))
    pred = P.Predictor(seed=4)
    # an arena of the predicted total, and one of 1000 slots that leaves
    # most updates to the overflow fill
    for budget in (0, 1000):
        keys = P.match_learned(t, dev(u_lo), dev(u_hi), pred, slot_budget=budget)
        torch.cuda.synchronize()
        assert_keys_equal(keys.cpu().numpy().view(np.uint64), want)
    t.free()
    pred.free()


@pytest.mark.parametrize("clustered", [False, True])
def test_segment_sort_size_classes(clustered):
    """Segments of every size class of the segment sort: 1, 2..16 (one lane),
    17..2048 (one wavefront, all six register widths), 2049..8192 (bitmap
    ranks of ids held in registers) and above (bitmap read back in order).
    With clustered ids (5000 consecutive ids share one box) the marks crowd
    into few bitmap entries."""
    rng = np.random.default_rng(19 + clustered)
    n = 100000
    s_lo = rng.uniform(0, 1e5, (1, n)).astype(np.float32)
    s_hi = (s_lo + np.float32(1.0)).astype(np.float32)
    if clustered:
        s_lo[0, 1000:6000] = np.float32(5e4)
        s_hi[0, 1000:6000] = np.float32(5e4 + 1)
    # query widths chosen to hit each class (about 2 boxes per unit length)
    widths = [0.0, 1.0, 10.0, 40.0, 100.0, 200.0, 400.0, 800.0, 2000.0, 5000.0, 12000.0, 30000.0]
    m = len(widths) * 8
    u_lo = rng.uniform(0, 1e5 - 6e4, (1, m)).astype(np.float32)
    u_lo[0, ::4] = np.float32(5e4 - 10.0)  # a quarter of them cover the cluster
    u_hi = (u_lo + np.repeat(np.asarray(widths, np.float32), 8)[None, :]).astype(np.float32)
    inst = W.Instance(s_lo, s_hi, u_lo, u_hi)
    want = oracle.itm(s_lo, s_hi, u_lo, u_hi, threads=8)
    cnt = oracle.counts_per_update(want, m)
    for lo, hi in [(2, 16), (17, 64), (65, 128), (129, 256), (257, 512), (513, 1024),
                   (1025, 2048), (2049, 16384), (16385, 1 << 30)]:
        assert ((cnt >= lo) & (cnt <= hi)).any(), (lo, hi, np.sort(cnt))
    for tr in TRAVERSALS:
        assert_keys_equal(gpu_match(inst, tr), want)


def test_empty_sets():
    import paper_1309_3458_amd as P
    torch = _torch()
    z = torch.zeros((2, 0), dtype=torch.float32, device="cuda")
    one = torch.ones((2, 5), dtype=torch.float32, device="cuda")
    t = P.build(z, z)
    assert P.match(t, one, one).numel() == 0
    t = P.build(one, one)
    assert P.match(t, z, z).numel() == 0
    keys = P.match(t, one, one)
    assert keys.numel() == 25


def test_tree_structure():
    import paper_1309_3458_amd as P
    inst = W.random_lengths(5, 100_003, 10, 3, L=1e5, max_len=500.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    n, d, H = t.info()
    assert (n, d) == (inst.n, 3) and (1 << H) - 1 >= n > (1 << (H - 1)) - 1
    for k in range(3):
        lo, hi, ids, mx = t.export(k)
        assert (np.diff(lo) >= 0).all()                        # in-order lower bounds
        assert np.array_equal(np.sort(ids), np.arange(n, dtype=np.uint32))
        np.testing.assert_array_equal(lo, inst.s_lo[k, ids])
        np.testing.assert_array_equal(hi, inst.s_hi[k, ids])
        # stable order: equal lower bounds keep increasing ids
        eq = lo[1:] == lo[:-1]
        assert (ids[1:][eq] > ids[:-1][eq]).all()
        # maxupper of every subtree, recomputed on the host
        P_ = (1 << H) - 1
        h_full = np.full(P_ + 1, -np.inf, np.float32)
        h_full[1:n + 1] = hi
        want = h_full.copy()
        for h in range(1, H):
            pos = np.arange(1 << h, P_ + 1, 1 << (h + 1))
            half = 1 << (h - 1)
            want[pos] = np.maximum(want[pos], np.maximum(want[pos - half], want[pos + half]))
        valid = np.array([max(1, p - (1 << (p & -p).bit_length() - 1) + 1) <= n
                          for p in range(1, P_ + 1)])
        np.testing.assert_array_equal(mx[valid], want[1:][valid])
    t.free()


@pytest.mark.parametrize("traversal", TRAVERSALS)
def test_counts_per_update(traversal):
    import paper_1309_3458_amd as P
    inst = W.uniform_instance(17, 40000, 30000, 2, 3000.0)
    want = oracle.counts_per_update(
        oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8), inst.m)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    cnt, K = P.count(t, dev(inst.u_lo), dev(inst.u_hi), traversal=traversal)
    np.testing.assert_array_equal(cnt.cpu().numpy().astype(np.uint32), want)
    assert K == int(want.sum())


def test_uniform_2d_1m_full_size():
    """The 1M-region, d=2, alpha=1 workload at full size: invariants, the
    closed-form pair count, and exact columns of M for sampled updates."""
    inst = W.uniform_2d_1m(1)
    got = gpu_match(inst, "auto")
    assert (np.diff(got.astype(np.int64)) > 0).all()
    EK = oracle.expected_pairs_uniform(inst.n, inst.m, [inst.side] * 2, W.L_SPACE)
    assert abs(len(got) - EK) <= 6 * np.sqrt(EK)
    rng = np.random.default_rng(123)
    sample = np.sort(rng.choice(inst.m, 4000, replace=False))
    sub = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo[:, sample], inst.u_hi[:, sample],
                     threads=8)
    # renumber the sampled columns back to their global update ids
    want = (sample[(sub >> np.uint64(32)).astype(np.int64)].astype(np.uint64) << np.uint64(32)) \
        | (sub & np.uint64(0xFFFFFFFF))
    upd = (got >> np.uint64(32)).astype(np.int64)
    mine = got[np.isin(upd, sample)]
    assert_keys_equal(mine, want)
    # both traversals agree everywhere
    assert_keys_equal(gpu_match(inst, "lane"), got)


def test_invalid_inputs_and_capacity():
    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    inst = W.uniform_instance(3, 1000, 1000, 2, 20000.0)
    s_lo = inst.s_lo.copy()
    s_lo[1, 17] = np.nan
    t = P.build(dev(s_lo), dev(inst.s_hi))
    with pytest.raises(N.DDMError) as e:
        P.match(t, dev(inst.u_lo), dev(inst.u_hi))
    assert e.value.code == N.DDM_E_INVALID_INPUT
    with pytest.raises(N.DDMError) as e:
        t.check()
    assert e.value.code == N.DDM_E_INVALID_INPUT
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    t.check()
    u_hi = inst.u_hi.copy()
    u_hi[0, 5] = inst.u_lo[0, 5] - 1.0   # lo > hi
    with pytest.raises(N.DDMError) as e:
        P.match(t, dev(inst.u_lo), dev(u_hi))
    assert e.value.code == N.DDM_E_INVALID_INPUT
    u_lo = inst.u_lo.copy()
    u_lo[1, 9] = np.inf
    with pytest.raises(N.DDMError) as e:
        P.match(t, dev(u_lo), dev(inst.u_hi))
    assert e.value.code == N.DDM_E_INVALID_INPUT
    # capacity: the exact count comes back, nothing is written
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    out = torch.full((len(want) - 1,), -7, dtype=torch.int64, device="cuda")
    with pytest.raises(N.DDMError) as e:
        P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out)
    assert e.value.code == N.DDM_E_CAPACITY and int(e.value.detail) == len(want)
    torch.cuda.synchronize()
    assert (out.cpu() == -7).all()
    out = torch.empty(len(want) + 10, dtype=torch.int64, device="cuda")
    K = P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out)
    assert K == len(want)
    assert_keys_equal(out[:K].cpu().numpy().view(np.uint64), want)
    # a later request on the same tree still succeeds
    assert_keys_equal(gpu_match(inst), want)


def test_bad_arguments():
    import ctypes
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    L = N.lib()
    x = torch.zeros((5, 10), dtype=torch.float32, device="cuda")
    h = ctypes.c_void_p()
    p = ctypes.c_void_p(x.data_ptr())
    assert L.ddm_build(p, p, 10, 0, None, ctypes.byref(h)) == N.DDM_E_INVALID_ARG
    assert L.ddm_build(p, p, 10, 5, None, ctypes.byref(h)) == N.DDM_E_INVALID_ARG
    assert L.ddm_build(None, None, 10, 2, None, ctypes.byref(h)) == N.DDM_E_INVALID_ARG
    assert L.ddm_build(p, p, 10, 2, None, None) == N.DDM_E_INVALID_ARG
    K = ctypes.c_uint64()
    assert L.ddm_match(None, p, p, 3, None, 0, ctypes.byref(K), None) == N.DDM_E_INVALID_ARG
    o = N.opts("tile")
    o.reserved[2] = 1
    assert L.ddm_build(p, p, 10, 2, None, ctypes.byref(h)) == N.DDM_OK
    assert L.ddm_match_ex(h, p, p, 10, None, 0, ctypes.byref(K), None,
                          ctypes.byref(o)) == N.DDM_E_INVALID_ARG
    o = N.opts("lane", 96)
    assert L.ddm_match_ex(h, p, p, 10, None, 0, ctypes.byref(K), None,
                          ctypes.byref(o)) == N.DDM_E_INVALID_ARG
    L.ddm_tree_free(h)
