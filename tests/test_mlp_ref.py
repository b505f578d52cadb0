"""Pins of the float64 predictor reference (test infrastructure for the GPU
training kernels): the analytic gradient against central finite differences,
and the feature estimate against exact counts."""
import numpy as np

import oracle
from oracle import mlp_ref
from paper_1309_3458_amd import workloads as W


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, mlp_ref.N_PARAMS)
    X = rng.normal(0, 1, (40, mlp_ref.N_IN))
    Y = rng.normal(0, 1, 40)
    L, g = mlp_ref.loss_grad(p, X, Y)
    assert abs(L - mlp_ref.loss(p, X, Y)) < 1e-12
    idx = rng.choice(mlp_ref.N_PARAMS, 200, replace=False)
    idx = np.concatenate([idx, [mlp_ref.N_PARAMS - 1, 0, 1152, 5312, 5376]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp_ref.loss(p + e, X, Y) - mlp_ref.loss(p - e, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_pack_unpack_roundtrip():
    p = np.arange(mlp_ref.N_PARAMS, dtype=np.float64)
    assert np.array_equal(mlp_ref.pack(*mlp_ref.unpack(p)), p)
    W1, b1, W2, b2, w3, b3 = mlp_ref.unpack(p)
    assert W1[1, 0] == 18 and b1[0] == 1152 and W2[0, 1] == 1217 and b3 == 5440


def test_feature_count_estimate_tracks_exact_counts():
    inst = W.uniform_instance(101, 20000, 3000, 2, 5000.0)
    X = mlp_ref.features(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    assert X.shape == (3000, 18)
    assert np.all(X[:, 10:15] == 0)              # dimension 2 absent
    for k in range(2):
        c = (np.searchsorted(np.sort(inst.s_lo[k]), inst.u_hi[k], side="right")
             - np.searchsorted(np.sort(inst.s_hi[k]), inst.u_lo[k], side="left"))
        est = X[:, 5 * k + 2] * inst.n
        # coarse histograms: the estimate follows the exact BITS count
        assert np.corrcoef(est, c)[0, 1] > 0.6
        assert abs(est.mean() - c.mean()) < 0.1 * c.mean()
    keys = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=4)
    K = oracle.counts_per_update(keys, inst.m)
    # joint corner estimate: for common sides it is the expected count
    est = np.expm1(X[:, 17] * 16)
    assert abs(est.mean() - K.mean()) < 0.15 * K.mean()
    assert np.corrcoef(est, K)[0, 1] > 0.3


def test_joint_estimate_follows_clusters():
    """On clustered boxes the joint lower-corner estimate tracks the exact
    per-update counts far better than the product of per-dimension ones."""
    inst = W.hotspot_2d(5, n=20000, m=4000)
    X = mlp_ref.features(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi)
    K = oracle.counts_per_update(
        oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=4), inst.m)
    est = np.expm1(X[:, 17] * 16)
    indep = inst.n * X[:, 2] * X[:, 7]
    good = K > 0
    e_joint = np.median(np.abs(np.log1p(est[good]) - np.log1p(K[good])))
    e_indep = np.median(np.abs(np.log1p(indep[good]) - np.log1p(K[good])))
    assert e_joint < 0.6 * e_indep


def test_corner_prefix_box_count_exact_on_cells():
    rng = np.random.default_rng(3)
    s_lo = rng.uniform(0, 1, (2, 500))
    H = mlp_ref._corner_prefix(s_lo, [0.0, 0.0], [1.0, 1.0], 8)
    # whole-cell boxes count exactly the corners inside them
    a = np.array([[2.0], [3.0]])
    b = np.array([[5.0], [7.0]])
    got = mlp_ref._box_count(H, a, b, 8)[0]
    cx = np.floor(s_lo[0] * 8)
    cy = np.floor(s_lo[1] * 8)
    want = np.sum((cx >= 2) & (cx < 5) & (cy >= 3) & (cy < 7))
    assert abs(got - want) < 1e-9


def test_features_hand_derived_1d():
    """Every feature of two updates on a 4-segment set, worked out by hand.

    S = [0,16], [16,32], [32,48], [48,64]: min lower 0, width 64, so the 64
    bins are the unit intervals and every edge an integer; mean length 16.
    Prefix counts: #lo < e is 1 for e in 1..16, 2 for 17..32, 3 for 33..48;
    the uppers fall in bins 16, 32, 48, 63, so #upper-bins < e is 0 up to 16,
    1 for 17..32.  Joint grid: 256 cells of width 1/4, lower corners in cells
    0, 64, 128, 192.
      U0 = [20, 40]: c = #lo<=40 (3) - #hi<20 (1) = 2; corner box
        [20-16, 40] -> cells [16, 160) hold 2 corners.
      U1 = [10, 16.5]: the interpolated #lo <= 16.5 is 1.5 (halfway between
        edge 16 with 1 and edge 17 with 2), #hi < 10 is 0: c = 1.5; corner
        box [-6, 16.5] -> cells [0, 66) hold 2 corners.
    """
    s_lo = np.array([[0, 16, 32, 48]], np.float32)
    s_hi = np.array([[16, 32, 48, 64]], np.float32)
    u_lo = np.array([[20, 10]], np.float32)
    u_hi = np.array([[40, 16.5]], np.float32)
    X = mlp_ref.features(s_lo, s_hi, u_lo, u_hi)
    want = np.zeros((2, 18))
    want[0, :5] = [20 / 64, 30 / 64, 2 / 4, np.log1p(2) / 16, 16 / 64]
    want[1, :5] = [6.5 / 64, 13.25 / 64, 1.5 / 4, np.log1p(1.5) / 16, 16 / 64]
    want[:, 15] = np.log2(4) / 20
    want[:, 16] = 1 / 3
    want[0, 17] = np.log1p(2) / 16
    want[1, 17] = np.log1p(2) / 16
    np.testing.assert_allclose(X, want, rtol=0, atol=1e-12)


def test_features_hand_derived_2d():
    """Two dimensions: the first as in the 1-D case; the second has lower
    bounds 0, 0, 32, 32 and uppers 32, 32, 64, 64 (width 64, mean length
    32).  U = [20,40] x [40,50]: second-dimension count #lo<=50 (4) -
    #hi-bins<40 (2) = 2; the joint grid has 64 cells per dimension (unit
    width), corners at cells (0,0), (16,0), (32,32), (48,32), and the corner
    box [4, 40) x [8, 50) holds only (32,32): estimate 1, which is also the
    exact count."""
    s_lo = np.array([[0, 16, 32, 48], [0, 0, 32, 32]], np.float32)
    s_hi = np.array([[16, 32, 48, 64], [32, 32, 64, 64]], np.float32)
    u_lo = np.array([[20], [40]], np.float32)
    u_hi = np.array([[40], [50]], np.float32)
    X = mlp_ref.features(s_lo, s_hi, u_lo, u_hi)
    want = np.zeros((1, 18))
    want[0, :5] = [20 / 64, 30 / 64, 2 / 4, np.log1p(2) / 16, 16 / 64]
    want[0, 5:10] = [10 / 64, 45 / 64, 2 / 4, np.log1p(2) / 16, 32 / 64]
    want[0, 15] = np.log2(4) / 20
    want[0, 16] = 2 / 3
    want[0, 17] = np.log1p(1) / 16
    np.testing.assert_allclose(X, want, rtol=0, atol=1e-12)
    assert oracle.itm(s_lo, s_hi, u_lo, u_hi).tolist() == [2]
