"""The count traversal's stash of hits (d > 1): when every hit fits, the
pairs are placed from the stash and no fill traversal runs; when the stash
overflows, the fill traversal runs.  Both give the oracle's keys bit for bit.
Which path ran is read from the library's kernel timing records."""
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


def _keys(t):
    return t.cpu().numpy().view(np.uint64)


def _paths(fn):
    import paper_1309_3458_amd as P
    P.prof_enable(True)
    P.prof_read()
    try:
        res = fn()
        rec = P.prof_read()
    finally:
        P.prof_enable(False)
    assert ("stash_scatter" in rec) <= ("traverse_tile_count_stash" in rec)
    return res, "stash_scatter" in rec, any(k.startswith("traverse_tile_fill") for k in rec)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_stash_holds_every_hit(d):
    """Few hits per update: the default stash holds them all."""
    import paper_1309_3458_amd as P
    inst = W.uniform_instance(900 + d, 40000, 30011, d, 2000.0 if d == 2 else 9000.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert len(want) > 0
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    got, stash, fill = _paths(lambda: P.match(t, dev(inst.u_lo), dev(inst.u_hi)))
    assert stash and not fill
    assert np.array_equal(_keys(got), want)
    torch = _torch()
    out = torch.full((len(want) + 5,), -7, dtype=torch.int64, device="cuda")
    k, stash, fill = _paths(lambda: P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out))
    assert k == len(want) and stash and not fill
    assert np.array_equal(_keys(out[:k]), want)
    assert bool((out[k:] == -7).all())
    t.free()


def test_stash_overflow_falls_back_to_fill():
    """Many hits per update: the default stash (sized from m) overflows and
    the fill traversal places the pairs; a capacity of more than 8 hits per
    update keeps no stash at all."""
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(910, 60000, 4001, 2, 60000.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert len(want) > 500 * inst.m
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    got, stash, fill = _paths(lambda: P.match(t, dev(inst.u_lo), dev(inst.u_hi)))
    assert fill and not stash
    assert np.array_equal(_keys(got), want)
    out = torch.empty(len(want), dtype=torch.int64, device="cuda")
    k, stash, fill = _paths(lambda: P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out))
    assert k == len(want) and fill and not stash
    assert np.array_equal(_keys(out), want)
    t.free()


def test_stash_exact_capacity_near_the_density_limit():
    """A capacity just under 8 hits per update sizes the stash exactly (a
    tile whose own slice of counted chunks is used up takes chunks from the
    next slices); the stash holds every hit."""
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(915, 60000, 40000, 2, 5600.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert 2 * inst.m < len(want) <= 8 * inst.m
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    out = torch.empty(len(want), dtype=torch.int64, device="cuda")
    k, stash, fill = _paths(lambda: P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out))
    assert k == len(want) and stash and not fill
    assert np.array_equal(_keys(out), want)
    t.free()


def test_stash_counts_and_ties():
    """Tie-heavy grids at every d > 1 through both entry points, and the
    per-update counts (which never stash)."""
    import paper_1309_3458_amd as P
    torch = _torch()
    for d in (2, 3, 4):
        inst = W.tiny_adversarial(920 + d, 3000, 2500, d)
        want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
        t = P.build(dev(inst.s_lo), dev(inst.s_hi))
        assert np.array_equal(_keys(P.match(t, dev(inst.u_lo), dev(inst.u_hi))), want)
        out = torch.empty(max(1, len(want)), dtype=torch.int64, device="cuda")
        k = P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out)
        assert np.array_equal(_keys(out[:k]), want)
        cnt, K = P.count(t, dev(inst.u_lo), dev(inst.u_hi))
        assert K == len(want)
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                              oracle.counts_per_update(want, inst.m).astype(np.int64))
        t.free()
