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
