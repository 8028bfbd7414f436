"""Pins of the FP64 warm-start network reference: convolution from its definition and the
backward pass by central finite differences."""
import numpy as np

from oracle import nn as R

TINY = R.NetConfig(m=15, s=8, conv_ch=(4, 4, 3), fc=(8, 6), nx=4, nt=3)


def _data(cfg, seed, B=2):
    rng = np.random.default_rng(seed)
    Xs, Ts, rs = [], [], []
    for _ in range(B):
        f = rng.standard_normal((cfg.s + 1, cfg.m))
        X, r = R.features(cfg, f, rng.uniform(0.5, 1.5, cfg.m), rng.uniform(0.5, 1.5, cfg.m),
                          rng.uniform(1.1, 1.9))
        Xs.append(X)
        Ts.append(rng.standard_normal(cfg.s * cfg.m))
        rs.append(r)
    return Xs, Ts, rs


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    L, C, Co, lout = 11, 3, 2, 6
    X = rng.standard_normal((L, C))
    W = rng.standard_normal((5 * C, Co))
    b = rng.standard_normal(Co)
    out = R.conv_forward(X, W, b, lout)
    for o in range(lout):
        for co in range(Co):
            acc = b[co]
            for t in range(5):
                i = 2 * o + t - 2
                if 0 <= i < L:
                    for c in range(C):
                        acc += X[i, c] * W[t * C + c, co]
            assert abs(out[o, co] - acc) < 1e-12


def test_parameter_count_and_synthesis_basis():
    assert TINY.num_params() == sum(k * n + n for k, n, *_ in TINY.layer_shapes())
    B = R.synthesis_basis(TINY)
    assert B.shape == (TINY.nx * TINY.nt, TINY.s * TINY.m)
    full = R.NetConfig(m=255, s=128)
    assert 1.8e6 < full.num_params() < 2.6e6


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(TINY.num_params()) * 0.3
    Xs, Ts, rs = _data(TINY, 2)
    loss, grad = R.loss_and_grad(TINY, theta, Xs, Ts, rs)
    assert np.isfinite(loss) and loss > 0
    h = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    fd = []
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd.append((R.loss_and_grad(TINY, tp, Xs, Ts, rs)[0] - R.loss_and_grad(TINY, tm, Xs, Ts, rs)[0]) / (2 * h))
    fd = np.array(fd)
    assert np.linalg.norm(grad[idx] - fd) <= 1e-6 * max(np.linalg.norm(fd), 1e-12)


def test_features_layout():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((TINY.s + 1, TINY.m))
    dp, dm = rng.uniform(size=TINY.m), rng.uniform(size=TINY.m)
    X, r = R.features(TINY, f, dp, dm, 1.7)
    assert abs(r - np.sqrt(np.mean(f ** 2))) < 1e-15
    np.testing.assert_allclose(X[:TINY.m, 0], f[0] / r)
    np.testing.assert_allclose(X[:TINY.m, TINY.s + 1], dp)
    assert np.all(X[TINY.m:] == 0) and np.allclose(X[:TINY.m, TINY.s + 3], 0.2)
