"""Float64 reference of the hit-count predictor -- TEST INFRASTRUCTURE ONLY.

Only the test suite may use this module.  It restates, in plain numpy with
float64 arithmetic, the network and the features that the GPU library
documents for its learned output sizing (not part of the paper's method):

  MLP 18 -> 64 -> 64 -> 1 with ReLU, parameters packed row-major as
  W1[64][18], b1[64], W2[64][64], b2[64], w3[64], b3 (5441 floats);
  loss = mean over samples of (yhat - y)^2.

Its analytic gradient is pinned against central finite differences in the
CPU test suite.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 18, 64
N_PARAMS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_HID + 1
BINS = 64


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == N_PARAMS
    o = 0
    W1 = p[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = p[o:o + N_HID]; o += N_HID
    W2 = p[o:o + N_HID * N_HID].reshape(N_HID, N_HID); o += N_HID * N_HID
    b2 = p[o:o + N_HID]; o += N_HID
    w3 = p[o:o + N_HID]; o += N_HID
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def forward(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def loss(p, X, Y):
    r = forward(p, X) - np.asarray(Y, dtype=np.float64)
    return float(np.mean(r * r))


def loss_grad(p, X, Y):
    """(loss, gradient) of the mean squared error by backpropagation."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    yhat = h2 @ w3 + b3
    r = yhat - Y
    dy = 2.0 * r / N
    gw3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return float(np.mean(r * r)), pack(gW1, gb1, gW2, gb2, gw3, gb3)


def _interp(c, u):
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lo = ~(u > 0)
    hi = u >= BINS
    mid = ~lo & ~hi
    b = np.floor(u[mid]).astype(np.int64)
    fr = u[mid] - b
    out[lo] = c[0]
    out[hi] = c[BINS]
    out[mid] = c[b] + fr * (c[b + 1] - c[b])
    return out


SAT_GRID = {1: 256, 2: 64, 3: 16}


def _corner_prefix(s_lo, mn, w, G):
    """(G+1)^d prefix counts of lower corners per grid cell (index + 1)."""
    d = s_lo.shape[0]
    cells = [np.clip(np.floor((s_lo[k] - mn[k]) / w[k] * G), 0, G - 1).astype(np.int64)
             for k in range(d)]
    H = np.zeros((G + 1,) * d)
    np.add.at(H, tuple(c + 1 for c in reversed(cells)), 1.0)   # axis 0 = last dim
    for ax in range(d):
        H = np.cumsum(H, axis=ax)
    return H


def _prefix_at(H, u, G):
    """Multilinear interpolation of the prefix array at grid point(s) u [d, m]."""
    d = u.shape[0]
    uu = np.clip(u, 0.0, G)
    i = np.minimum(np.floor(uu).astype(np.int64), G - 1)
    f = uu - i
    acc = np.zeros(u.shape[1])
    for c in range(1 << d):
        wgt = np.ones(u.shape[1])
        idx = []
        for k in range(d):
            hi = (c >> k) & 1
            wgt *= f[k] if hi else 1.0 - f[k]
            idx.append(i[k] + hi)
        acc += wgt * H[tuple(reversed(idx))]
    return acc


def _box_count(H, a, b, G):
    d = a.shape[0]
    tot = np.zeros(a.shape[1])
    for c in range(1 << d):
        pts = np.stack([b[k] if (c >> k) & 1 else a[k] for k in range(d)])
        neg = sum(0 if (c >> k) & 1 else 1 for k in range(d))
        v = _prefix_at(H, pts, G)
        tot += -v if neg % 2 else v
    return tot


def features(s_lo, s_hi, u_lo, u_hi):
    """Per-update features (d <= 3), float64, as documented by the library."""
    s_lo = np.asarray(s_lo, np.float64)
    s_hi = np.asarray(s_hi, np.float64)
    u_lo = np.asarray(u_lo, np.float64)
    u_hi = np.asarray(u_hi, np.float64)
    d, n = s_lo.shape
    m = u_lo.shape[1]
    X = np.zeros((m, N_IN))
    G = SAT_GRID[d]
    mns, ws, mes = [], [], []
    for k in range(d):
        mn = s_lo[k].min()
        mx = s_hi[k].max()
        w = max(mx - mn, 1e-30)
        edges = mn + w * np.arange(BINS + 1) / BINS
        edges[BINS] = mx
        slo = np.sort(s_lo[k])
        cum_lo = np.searchsorted(slo, edges, side="left").astype(np.float64)
        cum_lo[BINS] = np.searchsorted(slo, mx, side="right")
        b = np.clip(np.floor((s_hi[k] - mn) / w * BINS), 0, BINS - 1).astype(np.int64)
        cum_hi = np.concatenate([[0], np.cumsum(np.bincount(b, minlength=BINS))]).astype(np.float64)
        me = np.mean(s_hi[k] - s_lo[k])
        ql, qh = u_lo[k], u_hi[k]
        c_le = _interp(cum_lo, (qh - mn) / w * BINS)
        c_lt = _interp(cum_hi, (ql - mn) / w * BINS)
        c = np.clip(c_le - c_lt, 0.0, n)
        X[:, 5 * k + 0] = (qh - ql) / w
        X[:, 5 * k + 1] = (0.5 * (ql + qh) - mn) / w
        X[:, 5 * k + 2] = c / n
        X[:, 5 * k + 3] = np.log1p(c) / 16.0
        X[:, 5 * k + 4] = me / w
        mns.append(mn); ws.append(w); mes.append(me)
    H = _corner_prefix(s_lo, mns, ws, G)
    a = np.stack([(u_lo[k] - mes[k] - mns[k]) / ws[k] * G for k in range(d)])
    b = np.stack([(u_hi[k] - mns[k]) / ws[k] * G for k in range(d)])
    X[:, 15] = np.log2(n) / 20.0
    X[:, 16] = d / 3.0
    X[:, 17] = np.log1p(np.maximum(_box_count(H, a, b, G), 0.0)) / 16.0
    return X
