"""Sort-Based Matching on the GPU (Algorithm 3, the paper's sweep-line
comparison system), through the C ABI: bit-exact against the CPU oracle's
sweep (d = 1) and its brute force and ITM (every d), across several sweep
segments with ragged tails, exact ties, touching ends, points and signed
zeros, intervals that span every segment, ids above 2^20, empty sets,
invalid input and the capacity error."""
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


def _sbm(inst):
    import paper_1309_3458_amd as P
    return P.match_sbm(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo),
                       dev(inst.u_hi)).cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("n,m", [(1, 1), (63, 5), (64, 64), (65, 130), (1000, 333), (4097, 2049)])
def test_sbm_1d_equals_oracle_sweep(n, m):
    inst = W.tiny_adversarial(700 + n % 97, n, m, 1)
    want = oracle.sbm_1d(inst.s_lo[0], inst.s_hi[0], inst.u_lo[0], inst.u_hi[0])
    assert np.array_equal(_sbm(inst), want)
    assert np.array_equal(want, oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi))


@pytest.mark.parametrize("d", [2, 3, 4])
@pytest.mark.parametrize("n,m", [(1, 7), (129, 64), (3000, 700)])
def test_sbm_equals_oracle_brute(d, n, m):
    inst = W.tiny_adversarial(710 + 7 * d + n % 13, n, m, d)
    want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert np.array_equal(_sbm(inst), want)


@pytest.mark.parametrize("d", [1, 2])
def test_sbm_equals_itm_uniform_and_varlen(d):
    import paper_1309_3458_amd as P
    for inst in (W.uniform_instance(720 + d, 60000, 45001, d, 3000.0 if d == 2 else 40.0),
                 W.random_lengths(730 + d, 30011, 20000, d, max_len=60.0)):
        want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
        assert np.array_equal(_sbm(inst), want)
        t = P.build(dev(inst.s_lo), dev(inst.s_hi))
        itm = P.match(t, dev(inst.u_lo), dev(inst.u_hi)).cpu().numpy().view(np.uint64)
        t.free()
        assert np.array_equal(itm, want)


def test_sbm_spanning_intervals():
    """Subscriptions that cover the whole space sit in every segment's
    starting set; identical intervals tie on every key."""
    rng = np.random.default_rng(740)
    n, m = 5000, 900
    s_lo = rng.uniform(0, 1000, (1, n)).astype(np.float32)
    s_hi = (s_lo + rng.uniform(0, 5, (1, n))).astype(np.float32)
    s_lo[0, ::50], s_hi[0, ::50] = -1.0, 2000.0   # span everything
    s_lo[0, 1::97], s_hi[0, 1::97] = 500.0, 500.0  # one shared point
    u_lo = rng.uniform(0, 1000, (1, m)).astype(np.float32)
    u_hi = (u_lo + rng.uniform(0, 5, (1, m))).astype(np.float32)
    u_lo[0, :20], u_hi[0, :20] = 500.0, 500.0
    inst = W.Instance(s_lo, s_hi, u_lo, u_hi, name="span")
    want = oracle.sbm_1d(s_lo[0], s_hi[0], u_lo[0], u_hi[0])
    assert np.array_equal(_sbm(inst), want)


def test_sbm_ids_above_2_20():
    """More than 2^20 subscriptions: the per-update sort reads ids above the
    one-window bitmap from a copy."""
    inst = W.uniform_instance(750, (1 << 20) + 4099, 20000, 1, 60.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    assert len(want) > 0 and int(want.max() & 0xffffffff) >= (1 << 20)
    assert np.array_equal(_sbm(inst), want)


def test_sbm_edge_cases():
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_instance(760, 2000, 1500, 3, 20000.0)
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda")
    assert P.match_sbm(e, e, dev(inst.u_lo), dev(inst.u_hi)).numel() == 0
    assert P.match_sbm(dev(inst.s_lo), dev(inst.s_hi), e, e).numel() == 0
    bad = inst.s_hi.copy()
    bad[0, 77] = inst.s_lo[0, 77] - 1.0
    with pytest.raises(P.DDMError) as ex:
        P.match_sbm(dev(inst.s_lo), dev(bad), dev(inst.u_lo), dev(inst.u_hi))
    assert ex.value.code == -2
    badu = inst.u_lo.copy()
    badu[2, 5] = np.inf
    with pytest.raises(P.DDMError) as ex:
        P.match_sbm(dev(inst.s_lo), dev(inst.s_hi), dev(badu), dev(inst.u_hi))
    assert ex.value.code == -2
    want = oracle.brute(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert np.array_equal(_sbm(inst), want)
    small = torch.full((max(1, len(want) - 1),), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(P.DDMError) as ex:
        P.match_sbm(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi), out=small)
    assert ex.value.code == -3 and bool((small == -5).all())
