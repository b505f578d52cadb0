"""Dynamic DDM on the GPU (ddm_dynamic_*, through the C ABI): both sets and
both trees resident, extents of either set moved in rounds; after every
move the resident result equals a fresh ddm_build + ddm_match of the current
sets and the CPU oracle; invalid moves change nothing."""
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


def _fresh(s_lo, s_hi, u_lo, u_hi):
    import paper_1309_3458_amd as P
    t = P.build(dev(s_lo), dev(s_hi))
    k = P.match(t, dev(u_lo), dev(u_hi)).cpu().numpy().view(np.uint64)
    t.free()
    return k


@pytest.mark.parametrize("d,n,m,alpha", [(1, 3000, 2500, 20.0), (2, 20000, 15000, 5.0),
                                         (3, 8000, 9000, 30.0)])
def test_moves_equal_fresh_match_and_oracle(d, n, m, alpha):
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(600 + d, n, m, d, W.side_for_alpha(alpha, n + m, d))
    s_lo, s_hi = inst.s_lo.copy(), inst.s_hi.copy()
    u_lo, u_hi = inst.u_lo.copy(), inst.u_hi.copy()
    dy = P.Dynamic(dev(s_lo), dev(s_hi), dev(u_lo), dev(u_hi))
    want = oracle.itm(s_lo, s_hi, u_lo, u_hi, threads=8)
    assert np.array_equal(dy.pairs().cpu().numpy().view(np.uint64), want)
    rng = np.random.default_rng(610 + d)
    side = np.float32(inst.side)
    for rnd in range(6):
        which = rnd % 2  # subscriptions, then updates, alternately
        size = n if which == 0 else m
        c = int(rng.integers(1, max(2, size // 20)))
        if rnd == 4:
            c = size  # everything moves once
        ids = rng.choice(size, c, replace=False).astype(np.int32)
        lo = rng.uniform(0, 1e6, (d, c)).astype(np.float32)
        hi = (lo + side).astype(np.float32)
        if rnd == 2:
            hi[:, : c // 2] = lo[:, : c // 2]  # some points
        K = dy.move(which, dev(ids), dev(lo), dev(hi))
        if which == 0:
            s_lo[:, ids], s_hi[:, ids] = lo, hi
        else:
            u_lo[:, ids], u_hi[:, ids] = lo, hi
        got = dy.pairs().cpu().numpy().view(np.uint64)
        assert K == len(got)
        assert np.array_equal(got, _fresh(s_lo, s_hi, u_lo, u_hi)), f"round {rnd}"
        assert np.array_equal(got, oracle.itm(s_lo, s_hi, u_lo, u_hi, threads=8)), f"round {rnd}"
    dy.free()
    torch.cuda.synchronize()


def test_invalid_moves_change_nothing():
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(620, 5000, 4000, 2, 8000.0)
    dy = P.Dynamic(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi))
    before = dy.pairs().cpu().numpy()
    lo = np.full((2, 3), 10.0, np.float32)
    hi = np.full((2, 3), 20.0, np.float32)
    for which, ids in ((0, [1, 2, 1]), (1, [7, 8, 4000]), (0, [5000, 1, 2])):
        with pytest.raises(P.DDMError) as e:
            dy.move(which, dev(np.array(ids, np.int32)), dev(lo), dev(hi))
        assert e.value.code == P.DDM_E_INVALID_INPUT
    bad = hi.copy()
    bad[1, 1] = 5.0  # lo > hi
    with pytest.raises(P.DDMError) as e:
        dy.move(1, dev(np.array([1, 2, 3], np.int32)), dev(lo), dev(bad))
    assert e.value.code == P.DDM_E_INVALID_INPUT
    assert np.array_equal(dy.pairs().cpu().numpy(), before)
    # an empty move is a no-op
    assert dy.move(0, dev(np.zeros(0, np.int32)), dev(np.zeros((2, 0), np.float32)),
                   dev(np.zeros((2, 0), np.float32))) == len(before)
    dy.free()
    torch.cuda.synchronize()
