"""Moving subscriptions of a resident tree (ddm_tree_update, dynamic DDM),
through the C ABI: after the move, matching against the tree gives exactly
the oracle's pairs for the moved set; a move that keeps the trees' order is
refitted in place and leaves the tree identical (positions, ids, records,
maxupper) to a fresh build of the moved set; a move that breaks it rebuilds;
invalid moves change nothing."""
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


def _match(t, inst):
    import paper_1309_3458_amd as P
    return P.match(t, dev(inst.u_lo), dev(inst.u_hi)).cpu().numpy().view(np.uint64)


def _moved(inst, ids, nlo, nhi):
    s_lo, s_hi = inst.s_lo.copy(), inst.s_hi.copy()
    s_lo[:, ids] = nlo
    s_hi[:, ids] = nhi
    return W.Instance(s_lo, s_hi, inst.u_lo, inst.u_hi)


def _export(t, d):
    return [t.export(k) for k in range(d)]


def _same_export(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(np.asarray(u), np.asarray(v))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_refit_keeps_tree_identical_to_fresh_build(d):
    """Upper bounds grow or shrink, lower bounds move inside their gap: the
    (lower, id) order holds, so the tree is refitted."""
    import paper_1309_3458_amd as P
    rng = np.random.default_rng(40 + d)
    inst = W.uniform_instance(400 + d, 20000, 15000, d, 2000.0 if d > 1 else 50.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    ids = np.sort(rng.choice(inst.n, 700, replace=False)).astype(np.int32)
    nlo = inst.s_lo[:, ids].copy()
    # lower bounds of dimension 0 move a quarter of the way towards the next
    # lower bound in the tree (when that one does not move)
    order = np.lexsort((np.arange(inst.n), inst.s_lo[0]))
    rank = np.empty(inst.n, np.int64)
    rank[order] = np.arange(inst.n)
    nxt = order[np.minimum(rank[ids] + 1, inst.n - 1)]
    gap_lo = inst.s_lo[0, nxt].astype(np.float64)
    cand = (nlo[0] + 0.25 * (gap_lo - nlo[0])).astype(np.float32)
    ok = (rank[ids] + 1 < inst.n) & ~np.isin(nxt, ids) & (cand < inst.s_lo[0, nxt])
    nlo[0] = np.where(ok, cand, nlo[0])
    assert ok.sum() > 100
    nhi = (nlo + rng.uniform(0, 3000, nlo.shape)).astype(np.float32)
    rebuilt = t.update(dev(ids), dev(nlo), dev(nhi))
    assert rebuilt is False
    moved = _moved(inst, ids, nlo, nhi)
    want = oracle.itm(moved.s_lo, moved.s_hi, moved.u_lo, moved.u_hi, threads=8)
    assert np.array_equal(_match(t, moved), want)
    fresh = P.build(dev(moved.s_lo), dev(moved.s_hi))
    _same_export(_export(t, d), _export(fresh, d))
    t.free()
    fresh.free()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_large_moves_rebuild(d):
    import paper_1309_3458_amd as P
    rng = np.random.default_rng(50 + d)
    inst = W.uniform_instance(410 + d, 12000, 9000, d, 3000.0 if d > 1 else 80.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    for rnd in range(3):
        ids = rng.choice(inst.n, 1500, replace=False).astype(np.int32)
        nlo = rng.uniform(0, 1e6, (d, len(ids))).astype(np.float32)
        nhi = (nlo + rng.uniform(0, 5000, nlo.shape)).astype(np.float32)
        assert t.update(dev(ids), dev(nlo), dev(nhi)) is True
        inst = _moved(inst, ids, nlo, nhi)
        want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
        assert np.array_equal(_match(t, inst), want), f"round {rnd}"
    fresh = P.build(dev(inst.s_lo), dev(inst.s_hi))
    _same_export(_export(t, d), _export(fresh, d))
    t.free()


def test_invalid_moves_change_nothing():
    import paper_1309_3458_amd as P
    inst = W.uniform_instance(420, 5000, 4000, 2, 5000.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    before = _match(t, inst)
    ids = np.array([3, 17, 99], np.int32)
    nlo = inst.s_lo[:, ids].copy()
    nhi = inst.s_hi[:, ids].copy()
    nhi[1, 2] = nlo[1, 2] - 1.0
    with pytest.raises(P.DDMError) as e:
        t.update(dev(ids), dev(nlo), dev(nhi))
    assert e.value.code == -2
    with pytest.raises(P.DDMError) as e:
        t.update(dev(np.array([5000], np.int32)), dev(nlo[:, :1]), dev(inst.s_hi[:, :1]))
    assert e.value.code == -2
    assert np.array_equal(_match(t, inst), before)
    t.free()


def test_learned_match_after_update():
    """The learned-sizing statistics are recomputed after a move."""
    import paper_1309_3458_amd as P
    rng = np.random.default_rng(60)
    inst = W.uniform_instance(430, 20000, 20000, 2, 4000.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    pred = P.Predictor(5)
    P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), pred)  # statistics of the old set
    ids = rng.choice(inst.n, 4000, replace=False).astype(np.int32)
    nlo = rng.uniform(0, 2e5, (2, len(ids))).astype(np.float32)  # crowd one corner
    nhi = (nlo + np.float32(4000.0)).astype(np.float32)
    t.update(dev(ids), dev(nlo), dev(nhi))
    moved = _moved(inst, ids, nlo, nhi)
    got = P.match_learned(t, dev(moved.u_lo), dev(moved.u_hi), pred).cpu().numpy().view(np.uint64)
    want = oracle.itm(moved.s_lo, moved.s_hi, moved.u_lo, moved.u_hi, threads=8)
    assert np.array_equal(got, want)
    X = P.features(t, dev(moved.u_lo), dev(moved.u_hi)).cpu().numpy()
    from oracle import mlp_ref
    np.testing.assert_allclose(X, mlp_ref.features(moved.s_lo, moved.s_hi, moved.u_lo,
                                                   moved.u_hi), rtol=1e-3, atol=2e-4)
    t.free()
