"""Every configuration of the benchmark at full size, bit-exact against the
CPU oracle, in the launch configuration the benchmark times.

* d = 2, 500,000 + 500,000 squares of side 1000 (alpha = 1), seed 1: the
  whole sorted pair list of the plain two-pass path and of the learned
  single-pass path against the oracle's whole list;
* d = 2, 500,000 + 500,000 boxes around 16 Gaussian hotspots with
  log-normal sides (median 1e4), seed 2: about 1.8e9 pairs (14.6 GB) stay
  in device memory; 2,000 sampled updates' columns of M against the oracle,
  and the learned path's whole output equal to the plain path's, element by
  element on the device;
* the 256-instance batch (seed 3), one graph replay: every instance's slice
  against the oracle's whole list for that instance;
* the serving schedule (seed 4, d = 3, Poisson arrivals at 2,000 per second,
  N log-uniform in [1e3, 1e6]), its first second served in open loop with
  learned sizing: every 100th request against the oracle on up to 400 of its
  updates (each update's whole column of M);
* more than 2^20 subscriptions with segments above 16,384 keys: the segment
  sort that reads ids from a copy window by window, against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1309_3458_amd import workloads as W

pytestmark = pytest.mark.gpu

HOST_THREADS = 16


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _first_mismatch(got, want):
    assert got.shape == want.shape, (got.shape, want.shape)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"first mismatch at {bad[0]}: {got[bad[0]]:#x} vs {want[bad[0]]:#x}"


def _columns(keys_dev, sample):
    """The keys of the sampled updates (ascending ids) out of a sorted device
    key array, as uint64 on the host."""
    torch = _torch()
    lo = torch.from_numpy(sample.astype(np.int64) << 32).cuda()
    hi = torch.from_numpy((sample.astype(np.int64) + 1) << 32).cuda()
    a = torch.searchsorted(keys_dev, lo).cpu().numpy()
    b = torch.searchsorted(keys_dev, hi).cpu().numpy()
    parts = [keys_dev[int(x):int(y)].cpu().numpy().view(np.uint64) for x, y in zip(a, b)]
    return np.concatenate(parts) if parts else np.zeros(0, np.uint64)


def _oracle_columns(inst, sample, threads=HOST_THREADS):
    """The oracle's columns of M for the sampled updates, renumbered to their
    global update ids."""
    sub = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo[:, sample], inst.u_hi[:, sample],
                     threads=threads)
    j = sample[(sub >> np.uint64(32)).astype(np.int64)].astype(np.uint64)
    return (j << np.uint64(32)) | (sub & np.uint64(0xFFFFFFFF))


def _predictor():
    from paper_1309_3458_amd import learn
    pred, _ = learn.train_predictor(n_inst=16, per_instance=8000, epochs=10)
    return pred


def test_uniform_2d_1m_whole_list_plain_and_learned():
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.uniform_2d_1m(1)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=HOST_THREADS)
    EK = oracle.expected_pairs_uniform(inst.n, inst.m, [inst.side] * 2, W.L_SPACE)
    assert abs(len(want) - EK) <= 6 * np.sqrt(EK)
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
    out = torch.empty(len(want) + 1, dtype=torch.int64, device="cuda")
    t = P.build(s_lo, s_hi)
    got = P.match(t, u_lo, u_hi, out=out).cpu().numpy().view(np.uint64)
    _first_mismatch(got, want)
    pred = _predictor()
    info = {}
    got_l = P.match_learned(t, u_lo, u_hi, pred, out=out, info=info).cpu().numpy().view(np.uint64)
    _first_mismatch(got_l, want)
    assert info["slots"] > 0
    t.free()
    pred.free()
    torch.cuda.synchronize()


@pytest.mark.slow
def test_hotspot_2d_full_size_sampled_columns_and_learned_equal_plain():
    import paper_1309_3458_amd as P
    torch = _torch()
    inst = W.hotspot_2d(2)
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
    t = P.build(s_lo, s_hi)
    plain = P.match(t, u_lo, u_hi)
    K = plain.numel()
    assert K > 10 ** 9
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(inst.m, 2000, replace=False))
    _first_mismatch(_columns(plain, sample), _oracle_columns(inst, sample))
    # invariants over the whole list, on the device: strictly increasing
    # keys (no duplicates), every update id in range
    step = 1 << 28
    for a in range(0, K, step):
        blk = plain[a:min(K, a + step + 1)]
        assert bool((blk[1:] > blk[:-1]).all())
    assert int(plain[-1]) >> 32 < inst.m and int(plain[0]) >= 0
    pred = _predictor()
    info = {}
    learned = P.match_learned(t, u_lo, u_hi, pred, info=info)
    assert learned.numel() == K
    for a in range(0, K, step):
        assert torch.equal(learned[a:a + step], plain[a:a + step]), f"block at {a}"
    del learned, plain
    t.free()
    pred.free()
    torch.cuda.synchronize()


@pytest.mark.slow
def test_batch256_every_instance_against_the_oracle():
    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import tune
    torch = _torch()
    specs = W.batch_specs(3, 256)
    insts = [W.instance_from_spec(s) for s in specs]
    tens = [(dev(i.s_lo), dev(i.s_hi), dev(i.u_lo), dev(i.u_hi)) for i in insts]
    table = tune.Table.load(tune.DEFAULT_TABLE)
    qpts, wpc = table.qpts(specs), table.waves_per_cu
    K = tune.batch_total(tens, qpts)
    out = torch.empty(K, dtype=torch.int64, device="cuda")
    b = P.Batch(tens, K, qpts=qpts, waves_per_cu=wpc, use_graph=True, out=out)
    b.run()
    b.run()  # a replay of the captured graph, as the benchmark times it
    tot, rg = b.result()
    assert tot == K
    host = out[:tot].cpu().numpy().view(np.uint64)
    # the oracle's threads split each instance's updates (about 100 s of
    # host time on 16 cores for all 256 instances, most of it in the
    # largest d = 3 instances' per-dimension lists)
    for i, inst in enumerate(insts):
        want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=HOST_THREADS)
        got = host[int(rg[i]):int(rg[i + 1])]
        assert got.shape == want.shape and np.array_equal(got, want), \
            f"instance {i} ({inst.name})"
    b.free()
    torch.cuda.synchronize()


@pytest.mark.slow
def test_serving_schedule_first_second_every_100th_against_the_oracle():
    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import learn, serve
    torch = _torch()
    sched = W.serving_schedule(seed=4, rate=2000.0, duration_s=1.0, n_hi=1e6)
    assert len(sched) >= 1500
    pred, _ = learn.train_predictor(n_inst=16, per_instance=8000, epochs=10)
    srv = P.Server(predictor=pred, workers=8, host_pool=4 << 30)
    st = serve.run(srv, sched, sample_every=100, sample_max_pairs=1 << 31,
                   sample_bytes=16 << 30)
    srv.close()
    assert st["completed"] == len(sched) and st["n_errors"] == 0
    sampled = [i for i in range(0, len(sched), 100)]
    assert sorted(st["samples"]) == sampled
    rng = np.random.default_rng(4)
    for i in sampled:
        got = st["samples"][i]
        if isinstance(got, tuple):
            got = serve.keys_from_compact(*got)
        inst = W.Instance(*[x.cpu().numpy() for x in W.device_instance(sched[i].spec)])
        sample = np.arange(inst.m) if inst.m <= 400 else \
            np.sort(rng.choice(inst.m, 400, replace=False))
        upd = (got >> np.uint64(32)).astype(np.int64)
        _first_mismatch(got[np.isin(upd, sample)], _oracle_columns(inst, sample))
    pred.free()
    torch.cuda.synchronize()


def test_long_segments_over_2_pow_20_subscriptions():
    """n = 1.2e6 > 2^20 subscriptions (d = 1, length 10 on [0, 1e6)) and
    1,500 updates whose lengths give segments from a few keys to about
    36,000: the longest go to the bitmap sort, which reads the ids of
    in-place segments from a copy because they span two windows of 2^20."""
    import paper_1309_3458_amd as P
    torch = _torch()
    rng = np.random.default_rng(77)
    n, m = 1_200_000, 1_500
    s_lo = rng.uniform(0, 1e6, (1, n)).astype(np.float32)
    s_hi = (s_lo + np.float32(10.0)).astype(np.float32)
    u_lo = rng.uniform(0, 9.6e5, (1, m)).astype(np.float32)
    length = np.exp(rng.uniform(np.log(1.0), np.log(3.0e4), (1, m)))
    u_hi = (u_lo + length.astype(np.float32)).astype(np.float32)
    inst = W.Instance(s_lo, s_hi, u_lo, u_hi)
    want = oracle.itm(s_lo, s_hi, u_lo, u_hi, threads=HOST_THREADS)
    seg = np.bincount((want >> np.uint64(32)).astype(np.int64), minlength=m)
    assert seg.max() > 16384 and (seg > 2048).sum() > 100
    t = P.build(dev(s_lo), dev(s_hi))
    got = P.match(t, dev(u_lo), dev(u_hi)).cpu().numpy().view(np.uint64)
    t.free()
    _first_mismatch(got, want)
    # the same through the two-dimensional path (a second, wide dimension)
    lo2 = np.vstack([s_lo, np.zeros((1, n), np.float32)])
    hi2 = np.vstack([s_hi, np.full((1, n), 1.0, np.float32)])
    ul2 = np.vstack([u_lo, np.zeros((1, m), np.float32)])
    uh2 = np.vstack([u_hi, np.full((1, m), 1.0, np.float32)])
    t = P.build(dev(lo2), dev(hi2))
    got2 = P.match(t, dev(ul2), dev(uh2)).cpu().numpy().view(np.uint64)
    t.free()
    _first_mismatch(got2, want)
    torch.cuda.synchronize()
    del inst
