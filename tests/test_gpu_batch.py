"""Batched matching on the GPU (ddm_batch_*), through the C ABI.

* every instance's slice of the batch output is bit-exact against the CPU
  oracle (small batches of mixed d, n, m, alpha, full columns);
* the 256-instance batched workload at full size: every instance equals the
  single-instance matcher, sampled updates of several instances equal the
  oracle's columns of M;
* a captured graph replayed ten times, with other work and synchronizations
  in between, gives the eager bytes every time, also after the coordinates
  are overwritten in place;
* every work-item size and occupancy gives the same bytes;
* capacity and invalid-input errors write nothing and report the totals.
"""
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


def _tensors(insts):
    return [(dev(i.s_lo), dev(i.s_hi), dev(i.u_lo), dev(i.u_hi)) for i in insts]


def _batch(tens, capacity, **kw):
    import paper_1309_3458_amd as P
    return P.Batch(tens, capacity, **kw)


def _slices(b):
    torch = _torch()
    tot, rg = b.result()
    torch.cuda.synchronize()
    host = b.out[:tot].cpu().numpy().view(np.uint64)
    return [host[int(rg[i]):int(rg[i + 1])] for i in range(b.count)], tot


def _small_batch(seed, count, n_hi=2e4):
    specs = W.batch_specs(seed=seed, count=count, n_hi=n_hi)
    return [W.instance_from_spec(s) for s in specs]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_oracle(use_graph):
    insts = _small_batch(31, 20)
    want = [oracle.itm(i.s_lo, i.s_hi, i.u_lo, i.u_hi, threads=8) for i in insts]
    cap = sum(len(w) for w in want) + 17
    b = _batch(_tensors(insts), cap, use_graph=use_graph)
    b.run()
    got, tot = _slices(b)
    assert tot == cap - 17
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), f"instance {i} ({insts[i].name})"
    b.free()


def test_batch_edge_instances():
    """n or m of 1, ties and signed zeros (integer grid), every d, a mix of
    tile-sized and ragged update counts."""
    insts = [W.tiny_adversarial(40 + k, n, m, d) for k, (n, m, d) in enumerate(
        [(1, 1, 1), (1, 200, 2), (300, 1, 3), (64, 64, 4), (65, 129, 1), (2048, 2049, 2),
         (4097, 63, 3), (5000, 5000, 4)])]
    want = [oracle.itm(i.s_lo, i.s_hi, i.u_lo, i.u_hi, threads=8) for i in insts]
    b = _batch(_tensors(insts), sum(len(w) for w in want) + 1, use_graph=True)
    b.run()
    got, _ = _slices(b)
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), f"instance {i}"
    b.free()


@pytest.mark.parametrize("qpt,wpc", [(16, 1), (32, 4), (64, 24), (64, 64), (16, 0), (64, 0)])
def test_batch_work_item_sizes(qpt, wpc):
    insts = _small_batch(32, 12)
    want = [oracle.itm(i.s_lo, i.s_hi, i.u_lo, i.u_hi, threads=8) for i in insts]
    b = _batch(_tensors(insts), sum(len(w) for w in want), qpt=qpt, waves_per_cu=wpc)
    b.run()
    got, _ = _slices(b)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    b.free()


def test_graph_replays_equal_eager_and_follow_inputs():
    torch = _torch()
    insts = _small_batch(33, 16)
    tens = _tensors(insts)
    eager = _batch(tens, 50_000_000, use_graph=False)
    eager.run()
    ref, tot = _slices(eager)
    eager.free()
    g = _batch(tens, 50_000_000, use_graph=True)
    for r in range(10):
        g.run()
        got, t2 = _slices(g)
        assert t2 == tot
        for a, c in zip(got, ref):
            assert np.array_equal(a, c), f"replay {r}"
        # unrelated eager work and a synchronization between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
    # overwrite instance 0's updates in place: the replay reads the new values
    new = W.uniform_instance(99, insts[0].n, insts[0].m, insts[0].d, insts[0].side * 2.0)
    tens[0][2].copy_(dev(new.u_lo))
    tens[0][3].copy_(dev(new.u_hi))
    g.run()
    got, _ = _slices(g)
    w0 = oracle.itm(insts[0].s_lo, insts[0].s_hi, new.u_lo, new.u_hi, threads=8)
    assert np.array_equal(got[0], w0)
    for a, c in zip(got[1:], ref[1:]):
        assert np.array_equal(a, c)
    g.free()


def test_two_step_count_then_fill():
    """ddm_batch_count gives the total and ranges before any output exists;
    ddm_batch_fill then writes exactly the one-step bytes."""
    import paper_1309_3458_amd as P
    torch = _torch()
    insts = _small_batch(36, 10)
    want = [oracle.itm(i.s_lo, i.s_hi, i.u_lo, i.u_hi, threads=8) for i in insts]
    b = P.Batch(_tensors(insts), 0, use_graph=False)
    tot, rg = b.count_pairs()
    assert tot == sum(len(w) for w in want)
    assert np.array_equal(np.diff(rg.astype(np.int64)), [len(w) for w in want])
    out = torch.empty(tot, dtype=torch.int64, device="cuda")
    b.fill(out)
    torch.cuda.synchronize()
    host = out.cpu().numpy().view(np.uint64)
    for i, w in enumerate(want):
        assert np.array_equal(host[int(rg[i]):int(rg[i + 1])], w)
    # count again, then a fill that does not fit
    b.count_pairs()
    with pytest.raises(P.DDMError) as e:
        b.fill(out[: max(0, tot - 1)])
    assert e.value.code == -3
    b.free()
    g = P.Batch(_tensors(insts[:2]), 10 ** 7, use_graph=True)
    with pytest.raises(P.DDMError):
        g.count_pairs()
    g.free()


def test_capacity_and_invalid_input():
    import paper_1309_3458_amd as P
    torch = _torch()
    insts = _small_batch(34, 6)
    want = [oracle.itm(i.s_lo, i.s_hi, i.u_lo, i.u_hi, threads=8) for i in insts]
    K = sum(len(w) for w in want)
    tens = _tensors(insts)
    out = torch.full((K,), -7, dtype=torch.int64, device="cuda")
    b = P.Batch(tens, K - 1, out=out)
    b.run()
    with pytest.raises(P.DDMError) as e:
        b.result()
    assert e.value.code == -3
    assert b.total == K
    assert np.array_equal(np.diff(b._ranges.astype(np.int64)), [len(w) for w in want])
    assert bool((out == -7).all())
    b.free()
    # NaN in one instance: INVALID_INPUT, nothing written
    bad = [tuple(t.clone() for t in x) for x in tens]
    bad[3][0][0, 5] = float("nan")
    b = P.Batch(bad, K + 10, out=torch.full((K + 10,), -7, dtype=torch.int64, device="cuda"))
    b.run()
    with pytest.raises(P.DDMError) as e:
        b.result()
    assert e.value.code == -2
    assert bool((b.out == -7).all())
    b.free()
    # lo > hi in an update
    bad = [tuple(t.clone() for t in x) for x in tens]
    bad[1][2][0, 0] = 10.0
    bad[1][3][0, 0] = 9.0
    b = P.Batch(bad, K + 10, use_graph=False)
    b.run()
    with pytest.raises(P.DDMError):
        b.result()
    b.free()


def test_bad_batch_arguments():
    import paper_1309_3458_amd as P
    insts = _small_batch(35, 2)
    tens = _tensors(insts)
    with pytest.raises(P.DDMError):
        P.Batch(tens, 100, qpt=48)
    with pytest.raises(P.DDMError):
        P.Batch(tens, 100, waves_per_cu=65)
    with pytest.raises(P.DDMError):
        P.Batch([], 100)
    big = W.uniform_instance(5, 1 << 20, 10, 1, 1.0)
    with pytest.raises(P.DDMError):
        P.Batch(_tensors([big]), 100)


@pytest.mark.slow
def test_batched_workload_full_size():
    """The 256-instance batch (N log-uniform in [1e3, 2e5], d in {1,2,3},
    alpha log-uniform in [0.01, 100], seed 3) as the benchmark launches it:
    every instance equals the single-instance matcher; sampled updates of
    eight instances equal the oracle's columns of M."""
    import paper_1309_3458_amd as P
    torch = _torch()
    insts = W.batch_instances(3, 256)
    tens = _tensors(insts)
    singles = []
    for i, (a, b_, c, d_) in enumerate(tens):
        t = P.build(a, b_)
        singles.append(P.match(t, c, d_).cpu().numpy().view(np.uint64))
        t.free()
    K = sum(len(s) for s in singles)
    b = P.Batch(tens, K, use_graph=True)
    b.run()
    b.run()  # the replay, not only the capture run
    got, tot = _slices(b)
    assert tot == K
    for i, (g, s) in enumerate(zip(got, singles)):
        assert np.array_equal(g, s), f"instance {i} ({insts[i].name})"
    rng = np.random.default_rng(7)
    for i in rng.choice(len(insts), 8, replace=False):
        inst = insts[i]
        sample = np.sort(rng.choice(inst.m, min(inst.m, 300), replace=False))
        sub = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo[:, sample], inst.u_hi[:, sample],
                         threads=8)
        w = (sample[(sub >> np.uint64(32)).astype(np.int64)].astype(np.uint64) << np.uint64(32)) \
            | (sub & np.uint64(0xffffffff))
        upd = (got[i] >> np.uint64(32)).astype(np.int64)
        assert np.array_equal(got[i][np.isin(upd, sample)], w), f"instance {i}"
    b.free()
    torch.cuda.synchronize()


@pytest.mark.parametrize("use_graph", [False, True])
def test_sparse_batch_uses_the_stash(use_graph):
    """Few hits per update (alpha about 1, d = 2 and 3, plus d = 1 instances
    that the fill traversal writes): a capacity of at most 8 hits per update
    keeps the count traversal's hits, and the stash scatter places the
    pairs of the d > 1 instances; graph replays give the same bytes."""
    import paper_1309_3458_amd as P
    insts = []
    for i in range(12):
        d = (1, 2, 3)[i % 3]
        n, m = 3000 + 911 * i, 2000 + 677 * i
        insts.append(W.uniform_instance([920, i], n, m, d, W.side_for_alpha(1.0, n + m, d)))
    want = [oracle.itm(i.s_lo, i.s_hi, i.u_lo, i.u_hi, threads=8) for i in insts]
    K = sum(len(w) for w in want)
    M = sum(i.m for i in insts)
    assert 0 < K <= 8 * M
    b = _batch(_tensors(insts), K, use_graph=use_graph)
    P.prof_enable(True)
    P.prof_read()
    try:
        for r in range(3):
            b.run()
            got, tot = _slices(b)
            assert tot == K
            for i, (g, w) in enumerate(zip(got, want)):
                assert np.array_equal(g, w), f"run {r}, instance {i}"
        rec = P.prof_read()
    finally:
        P.prof_enable(False)
    if not use_graph:
        assert "batch_stash_scatter" in rec
    b.free()
