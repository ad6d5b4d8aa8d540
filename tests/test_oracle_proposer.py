"""Pins of the proposal-network oracle: loss against its closed form on a
degenerate network, gradients against central finite differences (a
different method), and Adam's first step against its known size."""
import math

import numpy as np

from paper_1907_12933_amd import inputs as I


def setup(B=40, F=6, H=9, seed=5):
    g = I.rng(seed)
    f = g.normal(size=(B, F))
    y = (g.random(B) < 0.3).astype(np.float64)
    W1 = g.normal(size=(H, F)) * 0.5
    b1 = g.normal(size=H) * 0.1
    w2 = g.normal(size=H) * 0.5
    return f, y, W1, b1, w2, 0.2


def test_loss_closed_form(orc):
    # W1 = 0, b1 = 0 -> s = c for every sample; loss = mean of the two log terms
    B, F, H = 7, 3, 4
    y = np.array([1, 0, 0, 1, 0, 0, 0], np.float64)
    c = 0.37
    r = orc.prop_loss_grad(np.ones((B, F)), y, 2.5, np.zeros((H, F)), np.zeros(H), np.ones(H), c)
    sig = 1 / (1 + math.exp(-c))
    exp = np.mean([-(2.5 * t * math.log(sig) + (1 - t) * math.log(1 - sig)) for t in y])
    assert abs(r["loss"] - exp) < 1e-14
    assert np.all(r["scores"] == c)


def test_gradients_finite_differences(orc):
    f, y, W1, b1, w2, c = setup()
    pw = 2.0
    r = orc.prop_loss_grad(f, y, pw, W1, b1, w2, c)
    h = 1e-6

    def loss(W1_, b1_, w2_, c_):
        return orc.prop_loss_grad(f, y, pw, W1_, b1_, w2_, c_)["loss"]

    for name, arr in (("W1", W1), ("b1", b1), ("w2", w2)):
        num = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            p = arr.copy(); p[idx] += h
            m = arr.copy(); m[idx] -= h
            args_p = dict(W1_=W1, b1_=b1, w2_=w2, c_=c); args_p[name + "_"] = p
            args_m = dict(W1_=W1, b1_=b1, w2_=w2, c_=c); args_m[name + "_"] = m
            num[idx] = (loss(**args_p) - loss(**args_m)) / (2 * h)
        err = np.linalg.norm(num - r[name]) / max(np.linalg.norm(num), 1e-30)
        assert err <= 1e-6, (name, err)
    numc = (loss(W1, b1, w2, c + h) - loss(W1, b1, w2, c - h)) / (2 * h)
    assert abs(numc - r["c"]) <= 1e-6 * max(abs(numc), 1e-12)


def test_adam_first_step(orc):
    # at t=1 the bias-corrected moments are g and g^2, so every parameter
    # moves by lr * g / (|g| + eps), i.e. by almost exactly lr against g
    g = np.array([0.5, -2.0, 1e-3, 0.0], np.float64)
    th = np.zeros(4); m = np.zeros(4); v = np.zeros(4)
    orc.adam_step(th, g, m, v, 1, lr=0.01, eps=1e-8)
    exp = -0.01 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(th, exp, rtol=1e-12, atol=0)
    assert abs(th[0] + 0.01) < 1e-9 and abs(th[1] - 0.01) < 1e-9 and th[3] == 0.0


def test_features_hand_built(orc):
    # 2x2 image, 3 first-layer units, shift 2 (window [0, 512)).
    # W1 rows (units) over pixels 0..3; x = (10, 0, 255, 100)
    W1 = np.array([[1, -2, 0, 3],
                   [-4, 0, 1, 1],
                   [2, 2, 2, 2]], np.int8)
    b1 = np.array([0, 100, -1000], np.int32)
    x = np.array([10, 0, 255, 100], np.uint8)
    # u = (10 + 300, -40 + 255 + 100 + 100, 20 + 510 + 200 - 1000) = (310, 415, -270)
    # live (0 <= u < 512): units 0 and 1
    net = I.QNet([4, 3, 2], [W1, np.ones((2, 3), np.int8)], [b1, np.zeros(2, np.int32)], [2])
    D = np.array([-20, 5], np.int16)
    f = orc.prop_features(net, x, 2, 2, D)
    assert f.shape == (8, 32)
    n1 = np.array([7, 4, 3, 6], float)
    n2 = np.sqrt(np.array([21, 8, 5, 14], float))
    nl = np.array([5, 2, 1, 4], float)
    for p in range(4):
        for i, d in enumerate(D):
            row = f[p * 2 + i]
            e = min(max(int(x[p]) + int(d), 0), 255) - int(x[p])
            assert np.allclose(row[:9], [p // 2, p % 2, x[p] / 255, d / 20, e / 20,
                                         n1[p] / 7, n2[p] / np.sqrt(21), nl[p] / 7, 1.0])
            assert np.all(row[9:] == 0)
    # clamping: pixel 2 (255) with +5 has e = 0; pixel 1 (0) with -20 has e = 0
    assert f[2 * 2 + 1][4] == 0 and f[1 * 2 + 0][4] == 0
