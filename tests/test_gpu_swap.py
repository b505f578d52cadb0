"""Tree on the smaller set (the n <= m role swap of Sec. IV), through the
C ABI: whatever the policy, the keys are bit-identical to the oracle's and
to build(S) + match(U); covers n > m and n < m, every d, update counts whose
ids need one, two and three radix digits, ties, empty sets, invalid input in
either set and the capacity error."""
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


def _sets(inst, policy):
    import paper_1309_3458_amd as P
    keys, sw = P.match_sets(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi),
                            swap=policy, return_swapped=True)
    return keys.cpu().numpy().view(np.uint64), sw


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("n,m", [(1, 1), (300, 1), (900, 200), (200, 900), (5000, 257)])
def test_swap_policies_equal_oracle(d, n, m):
    import paper_1309_3458_amd as P
    inst = W.tiny_adversarial(800 + 5 * d + n % 17 + m % 7, n, m, d)
    want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    for policy in (P.SWAP_AUTO, P.SWAP_NEVER, P.SWAP_ALWAYS):
        got, sw = _sets(inst, policy)
        assert np.array_equal(got, want), policy
        assert sw == (policy == P.SWAP_ALWAYS or (policy == P.SWAP_AUTO and n > m and d >= 3))


@pytest.mark.parametrize("m", [200, 70000])
def test_swap_uniform_large(m):
    """n > m at sizes spanning many tiles; 70000 updates need three digits.
    At d = 2 the default keeps the tree on the subscriptions."""
    import paper_1309_3458_amd as P
    inst = W.uniform_instance(820 + m % 5, 200003, m, 2, 2500.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    got, sw = _sets(inst, P.SWAP_ALWAYS)
    assert sw and np.array_equal(got, want)
    got, sw = _sets(inst, P.SWAP_AUTO)
    assert not sw and np.array_equal(got, want)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    plain = P.match(t, dev(inst.u_lo), dev(inst.u_hi)).cpu().numpy().view(np.uint64)
    t.free()
    assert np.array_equal(plain, want)


def test_swap_edge_cases():
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(830, 3000, 700, 3, 20000.0)
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda")
    for policy in (P.SWAP_AUTO, P.SWAP_ALWAYS):
        assert P.match_sets(e, e, dev(inst.u_lo), dev(inst.u_hi), swap=policy).numel() == 0
        assert P.match_sets(dev(inst.s_lo), dev(inst.s_hi), e, e, swap=policy).numel() == 0
    bad = inst.s_hi.copy()
    bad[1, 9] = np.nan
    badu = inst.u_lo.copy()
    badu[0, 3] = inst.u_hi[0, 3] + 1.0
    for policy in (P.SWAP_AUTO, P.SWAP_NEVER, P.SWAP_ALWAYS):
        with pytest.raises(P.DDMError) as ex:
            P.match_sets(dev(inst.s_lo), dev(bad), dev(inst.u_lo), dev(inst.u_hi), swap=policy)
        assert ex.value.code == -2
        with pytest.raises(P.DDMError) as ex:
            P.match_sets(dev(inst.s_lo), dev(inst.s_hi), dev(badu), dev(inst.u_hi), swap=policy)
        assert ex.value.code == -2
    want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert len(want) > 1
    small = torch.full((len(want) - 1,), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(P.DDMError) as ex:
        P.match_sets(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi), out=small)
    assert ex.value.code == -3 and bool((small == -5).all())
    with pytest.raises(P.DDMError) as ex:
        P.match_sets(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi), swap=7)
    assert ex.value.code == -1
