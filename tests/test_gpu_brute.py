"""Brute-Force Matching on the GPU (Algorithm 2, the paper's baseline),
through the C ABI: bit-exact against the CPU oracle's brute force and ITM,
across chunk boundaries of the staged subscriptions, ragged update counts,
every d, empty sets, invalid input and the capacity error."""
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


def _brute(inst):
    import paper_1309_3458_amd as P
    return P.match_brute(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo),
                         dev(inst.u_hi)).cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("n,m", [(1, 1), (1023, 255), (1024, 257), (1025, 64), (3000, 700)])
def test_brute_equals_oracle(d, n, m):
    inst = W.tiny_adversarial(500 + 7 * d + n % 11, n, m, d)
    want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert np.array_equal(_brute(inst), want)


def test_brute_equals_itm_uniform():
    import paper_1309_3458_amd as P
    inst = W.uniform_instance(510, 50000, 40000, 2, 3000.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    itm = P.match(t, dev(inst.u_lo), dev(inst.u_hi)).cpu().numpy().view(np.uint64)
    t.free()
    assert np.array_equal(_brute(inst), itm)
    assert np.array_equal(itm, oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8))


def test_brute_edge_cases():
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(511, 2000, 1500, 3, 20000.0)
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda")
    assert P.match_brute(e, e, dev(inst.u_lo), dev(inst.u_hi)).numel() == 0
    assert P.match_brute(dev(inst.s_lo), dev(inst.s_hi), e, e).numel() == 0
    bad = inst.s_lo.copy()
    bad[1, 77] = np.nan
    with pytest.raises(P.DDMError) as ex:
        P.match_brute(dev(bad), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi))
    assert ex.value.code == -2
    badu = inst.u_hi.copy()
    badu[2, 5] = inst.u_lo[2, 5] - 1.0
    with pytest.raises(P.DDMError) as ex:
        P.match_brute(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(badu))
    assert ex.value.code == -2
    want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    small = torch.full((max(1, len(want) - 1),), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(P.DDMError) as ex:
        P.match_brute(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi), out=small)
    assert ex.value.code == -3 and bool((small == -5).all())
