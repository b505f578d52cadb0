"""Update order and sort configurations that only change the work, never the
pairs: bimodal update extents (the sampled cell shape suits one mode, the
other mode's updates share cell buckets with it), extents on both sides of
the 1-D / cell threshold, and tree builds whose sort runs either tile size
(4096-key tiles while one per compute unit covers the arrays, 8192-key tiles
beyond).  Pair keys and counts are compared with the CPU oracle bit for bit.
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


def _keys(t):
    return t.cpu().numpy().view(np.uint64)


def _bimodal(seed, n, m, d, small, large):
    """Uniform corners in [0, L)^d; subscriptions and the first half of the
    updates have side `small`, the other updates side `large`."""
    rng = np.random.default_rng(seed)
    L = W.L_SPACE

    def boxes(count, side):
        lo = rng.uniform(0.0, L, size=(d, count)).astype(np.float32)
        hi = (lo + np.asarray(side, np.float32)).astype(np.float32)
        return lo, hi

    s_lo, s_hi = boxes(n, small)
    side = np.where(np.arange(m) < m // 2, small, large).astype(np.float32)
    u_lo, u_hi = boxes(m, side[None, :])
    return W.Instance(s_lo, s_hi, np.ascontiguousarray(u_lo), np.ascontiguousarray(u_hi),
                      name="bimodal")


@pytest.mark.parametrize("d", [2, 3, 4])
def test_bimodal_extents_equal_oracle(d):
    import paper_1309_3458_amd as P
    torch = _torch()
    n, m = (60000, 40000) if d < 4 else (40000, 24000)
    small = W.side_for_alpha(1.0, n + m, d)
    inst = _bimodal(700 + d, n, m, d, small, {2: 12.0, 3: 4.0, 4: 2.5}[d] * small)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert len(want) > m
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    got = _keys(P.match(t, dev(inst.u_lo), dev(inst.u_hi)))
    assert np.array_equal(got, want)
    out = torch.empty(len(want), dtype=torch.int64, device="cuda")
    k = P.match_into(t, dev(inst.u_lo), dev(inst.u_hi), out)
    assert k == len(want) and np.array_equal(_keys(out), want)
    cnt, K = P.count(t, dev(inst.u_lo), dev(inst.u_hi))
    assert K == len(want)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                          oracle.counts_per_update(want, m).astype(np.int64))
    t.free()


@pytest.mark.parametrize("factor", [0.25, 1.0, 4.0, 16.0])
def test_extents_around_the_cell_threshold(factor):
    """Candidate ranges from about 60 to about 4000 positions, so that the
    updates take 1-D buckets, cells, or a mix of both."""
    import paper_1309_3458_amd as P
    n, m = 120000, 30000
    side = W.side_for_alpha(1.0, 1_000_000, 2) * factor
    inst = W.uniform_instance(710 + int(factor * 4), n, m, 2, side)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    got = _keys(P.match(t, dev(inst.u_lo), dev(inst.u_hi)))
    t.free()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [300_000, 1_200_000])
def test_tree_sort_tile_sizes(n):
    """d = 3 trees of 300,000 (3 x 74 tiles of 4096 keys: one per compute
    unit) and 1,200,000 subscriptions (3 x 293 tiles: 8192-key tiles, more
    than the device holds at once); every pair equals the oracle's."""
    import paper_1309_3458_amd as P
    d, m = 3, 3000
    side = W.side_for_alpha(1.0, 1_000_000, d)
    inst = W.uniform_instance(720 + n % 7, n, m, d, side)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    got = _keys(P.match(t, dev(inst.u_lo), dev(inst.u_hi)))
    t.free()
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert np.array_equal(got, want)
