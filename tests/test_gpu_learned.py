"""Learned output sizing on the GPU, through the C ABI.

* the network's forward pass, gradient and Adam step against the float64
  reference (gradient within relative 1e-4);
* the per-update features against their float64 restatement;
* the single-pass matcher returns exactly the bytes of the plain matcher for
  trained, untrained, forced-zero-capacity and tiny-arena predictors, with
  both traversal kernels;
* training lowers the loss, and the trained network overflows far fewer
  updates than an untrained one on a shifted (hotspot) distribution;
* the predictor file round trip (ddm_predictor_save / ddm_predictor_load)
  and the refusal of damaged files.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp_ref
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


@pytest.fixture(scope="module")
def trained():
    _torch()
    from paper_1309_3458_amd import learn
    p, rep = learn.train_predictor(n_inst=16, per_instance=8000, epochs=12)
    return p, rep


def test_forward_matches_reference():
    import paper_1309_3458_amd as P
    rng = np.random.default_rng(1)
    params = rng.normal(0, 0.25, mlp_ref.N_PARAMS).astype(np.float32)
    X = rng.normal(0, 1, (3001, 18)).astype(np.float32)
    p = P.Predictor(3)
    p.set_params(params, 0.0)
    got = p.forward(dev(X)).cpu().numpy()
    want = mlp_ref.forward(params.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(got - want)) <= 1e-4 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("N", [1, 127, 128, 1000, 4097])
def test_gradient_matches_reference(N):
    import paper_1309_3458_amd as P
    rng = np.random.default_rng(N)
    params = rng.normal(0, 0.25, mlp_ref.N_PARAMS).astype(np.float32)
    X = rng.normal(0, 1, (N, 18)).astype(np.float32)
    Y = rng.normal(0, 1, N).astype(np.float32)
    p = P.Predictor(0)
    p.set_params(params, 0.0)
    g, loss = p.grad(dev(X), dev(Y))
    g = g.cpu().numpy().astype(np.float64)
    L, gref = mlp_ref.loss_grad(params.astype(np.float64), X.astype(np.float64),
                                Y.astype(np.float64))
    scale = np.max(np.abs(gref))
    err = np.abs(g - gref)
    assert np.all(err <= 1e-4 * np.abs(gref) + 1e-6 * scale), np.max(err / (np.abs(gref) + 1e-30))
    assert abs(float(loss.cpu()[0]) - L) <= 1e-4 * L


def test_adam_step_matches_reference():
    import paper_1309_3458_amd as P
    rng = np.random.default_rng(5)
    params = rng.normal(0, 0.25, mlp_ref.N_PARAMS).astype(np.float32)
    grads = [rng.normal(0, 0.1, mlp_ref.N_PARAMS).astype(np.float32) for _ in range(3)]
    p = P.Predictor(0)
    p.set_params(params, 0.0)
    m1 = np.zeros(mlp_ref.N_PARAMS)
    m2 = np.zeros(mlp_ref.N_PARAMS)
    th = params.astype(np.float64)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for t, g in enumerate(grads, 1):
        p.adam(dev(g), lr)
        m1 = b1 * m1 + (1 - b1) * g
        m2 = b2 * m2 + (1 - b2) * g.astype(np.float64) ** 2
        th = th - lr * (m1 / (1 - b1 ** t)) / (np.sqrt(m2 / (1 - b2 ** t)) + eps)
    got, _ = p.params()
    np.testing.assert_allclose(got, th, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_features_match_reference(d):
    import paper_1309_3458_amd as P
    inst = W.random_lengths(200 + d, 30000, 5000, d, L=1e5, max_len=800.0)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    X = P.features(t, dev(inst.u_lo), dev(inst.u_hi)).cpu().numpy()
    ref = mlp_ref.features(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert X.shape == ref.shape
    np.testing.assert_allclose(X, ref, rtol=1e-3, atol=2e-4)


def _plain(inst, traversal="auto"):
    import paper_1309_3458_amd as P
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    return t, P.match(t, dev(inst.u_lo), dev(inst.u_hi), traversal=traversal).cpu().numpy()


CASES = [
    W.uniform_instance(300, 60000, 50000, 2, 3000.0),
    W.uniform_instance(301, 30000, 40000, 3, 20000.0),
    W.hotspot_2d(302, n=40000, m=30000),
    W.random_lengths(303, 20000, 20000, 2, L=2e4, max_len=400.0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("traversal", ["tile", "lane"])
def test_learned_equals_plain(trained, case, traversal):
    import paper_1309_3458_amd as P
    p, _ = trained
    inst = CASES[case]
    t, want = _plain(inst, traversal)
    info = {}
    got = P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), p, traversal=traversal,
                          info=info).cpu().numpy()
    assert np.array_equal(got, want)
    assert info["overflowed"] <= inst.m
    # a tiny fixed arena: most updates overflow by arena, same bytes
    info = {}
    got = P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), p, slot_budget=1000,
                          traversal=traversal, info=info).cpu().numpy()
    assert np.array_equal(got, want)
    assert info["budget"] == 1000


def test_forced_under_prediction_falls_back(trained):
    """Capacities forced to 0 (delta = -30): every update with a hit takes the
    plain fill, and the bytes are unchanged."""
    import paper_1309_3458_amd as P
    p, _ = trained
    params, delta = p.params()
    q = P.Predictor(0)
    q.set_params(params, -30.0)
    inst = CASES[0]
    t, want = _plain(inst)
    info = {}
    got = P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), q, info=info).cpu().numpy()
    assert np.array_equal(got, want)
    K = oracle.counts_per_update(want.view(np.uint64) if want.dtype != np.uint64 else want,
                                 inst.m)
    assert info["slots"] == 0 and info["overflowed"] == int((K > 0).sum())


def test_oracle_parity_of_learned_path(trained):
    import paper_1309_3458_amd as P
    p, _ = trained
    inst = W.uniform_instance(310, 8000, 7000, 3, 30000.0)
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    got = P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), p).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)


def test_training_gain_over_untrained(trained):
    """What the trained network buys: on hotspot data (a shifted distribution)
    it overflows far fewer updates than the untrained network, whose slots
    are essentially arbitrary."""
    import paper_1309_3458_amd as P
    p, rep = trained
    assert rep["loss_last"] < 0.5 * rep["loss_first"]
    assert rep["val_under_rate"] <= 0.02
    inst = W.hotspot_2d(320, n=50000, m=50000)
    t = P.build(dev(inst.s_lo), dev(inst.s_hi))
    raw = P.Predictor(77)
    i_raw, i_tr = {}, {}
    a = P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), raw, info=i_raw).cpu().numpy()
    b = P.match_learned(t, dev(inst.u_lo), dev(inst.u_hi), p, info=i_tr).cpu().numpy()
    assert np.array_equal(a, b)
    assert i_tr["overflowed"] < 0.25 * max(1, i_raw["overflowed"])
    assert i_tr["overflowed"] < 0.2 * inst.m


@pytest.mark.slow
def test_learned_gain_over_plain_on_hotspots():
    """What the learned single pass gains over the plain two-pass path on the
    hotspot workload (500,000 + 500,000 boxes around 16 Gaussian hotspots,
    log-normal sides, seed 2; about 1.8e9 pairs): the same bytes, no count
    traversal (one pass over tiles cut by predicted work), and a shorter
    build + match step (median of 3 timed steps each, after a warm-up)."""
    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import learn
    torch = _torch()
    pred, _ = learn.train_predictor(n_inst=32, per_instance=16000, epochs=20)
    inst = W.hotspot_2d(2)
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
    t = P.build(s_lo, s_hi)
    plain = P.match(t, u_lo, u_hi)
    K = plain.numel()
    learned = torch.empty_like(plain)
    P.match_learned(t, u_lo, u_hi, pred, out=learned)
    t.free()
    assert torch.equal(learned, plain)
    del learned

    def step(path):
        tt = P.build(s_lo, s_hi)
        if path == "plain":
            k = P.match(tt, u_lo, u_hi, out=plain).numel()
        else:
            k = P.match_learned(tt, u_lo, u_hi, pred, out=plain).numel()
        tt.free()
        return k

    kernels, ms = {}, {}
    for path in ("plain", "learned"):
        step(path)
        P.prof_enable(True)
        P.prof_read()
        assert step(path) == K
        torch.cuda.synchronize()
        kernels[path] = P.prof_read()
        P.prof_enable(False)
        times = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            assert step(path) == K
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms[path] = sorted(times)[1]
    assert any(k.startswith("traverse_tile_count") for k in kernels["plain"])
    assert not any(k.startswith("traverse_tile_count") for k in kernels["learned"])
    assert "traverse_tile_fill_balanced" in kernels["learned"]
    print(f"hotspot step: plain {ms['plain']:.2f} ms, learned {ms['learned']:.2f} ms")
    assert ms["learned"] < ms["plain"], ms
    pred.free()


def test_predictor_file_round_trip(trained, tmp_path):
    """ddm_predictor_save / ddm_predictor_load: the loaded predictor has the
    same parameters and delta bit for bit and gives the same forward pass;
    a truncated file, another format and a missing file are refused."""
    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    p, _ = trained
    path = str(tmp_path / "pred.ddmp")
    p.save(path)
    q = P.Predictor.load(path)
    a, da = p.params()
    b, db = q.params()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)) and np.float32(da) == np.float32(db)
    X = torch.randn(300, 18, device="cuda")
    assert torch.equal(p.forward(X), q.forward(X))
    q.free()
    raw = open(path, "rb").read()
    assert raw[:4] == b"DDMP" and len(raw) == 16 + 4 * 5441
    bad = tmp_path / "bad.ddmp"
    for blob in (raw[:-4], raw + b"\0", b"XXXX" + raw[4:]):
        bad.write_bytes(blob)
        with pytest.raises(P.DDMError) as e:
            P.Predictor.load(str(bad))
        assert e.value.code == N.DDM_E_INVALID_INPUT
    with pytest.raises(P.DDMError) as e:
        P.Predictor.load(str(tmp_path / "missing.ddmp"))
    assert e.value.code == N.DDM_E_INVALID_ARG


def test_prepare_learned_moves_the_statistics_out_of_the_match():
    """ddm_tree_prepare_learned: the first learned match on a fresh tree
    computes the features' statistics; after prepare_learned it computes
    none and returns the same bytes (equal to the oracle).  Calling it twice
    is harmless; d = 4 and an empty set are refused."""
    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import _native as N
    torch = _torch()
    inst = W.uniform_instance(41, 12000, 9000, 2, W.side_for_alpha(5.0, 21000, 2))
    want = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=8)
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
    pred = P.Predictor(seed=6)
    ran = {}
    for prepared in (False, True):
        t = P.build(s_lo, s_hi)
        if prepared:
            t.prepare_learned()
            t.prepare_learned()
        torch.cuda.synchronize()
        P.prof_enable(True)
        P.prof_read()
        keys = P.match_learned(t, u_lo, u_hi, pred)
        torch.cuda.synchronize()
        ran[prepared] = P.prof_read()
        P.prof_enable(False)
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), want)
        t.free()
    assert "feature_stats" in ran[False]
    assert "feature_stats" not in ran[True]
    pred.free()
    for lo, hi in ((torch.zeros((4, 10), device="cuda"), torch.ones((4, 10), device="cuda")),
                   (torch.zeros((2, 0), device="cuda"), torch.zeros((2, 0), device="cuda"))):
        t = P.build(lo, hi)
        with pytest.raises(P.DDMError) as e:
            t.prepare_learned()
        assert e.value.code == N.DDM_E_INVALID_ARG
        t.free()
