"""Pins of the oracle's training loss and gradient (the networks are trained
on labelled examples by backpropagation, Sec. II-A; the paper adds the
verifier's counterexamples to the training set, Sec. VI):

  - the gradient against central finite differences of the loss, in every
    coordinate of theta (every W and b of every layer), on two networks;
  - closed forms: all-zero weights give loss log(C) and bias gradient
    (1/C - onehot) averaged; one layer (no hidden unit) is multinomial
    logistic regression, loss = scikit-learn's log_loss of the softmax and
    gradient = (p - onehot)^T [x/256, 1] / n;
  - a hidden layer with zero first-layer weights feeds the constant
    sigmoid(b_1) (scipy's expit) to the logits;
  - invariants: shifting every last-layer bias by one constant leaves the
    loss unchanged, and the last-layer bias gradient sums to zero;
  - Adam: its first step moves every parameter with a nonzero gradient by
    lr against the gradient's sign (bias-corrected m / sqrt(v) = g / |g|),
    and training on a separable set drives the loss down."""
import numpy as np
import pytest
from scipy.special import expit, softmax

from paper_1907_12933_amd import inputs as I


def f64net(dims, g, scale=0.7):
    W = [g.normal(0, scale, size=(dims[l + 1], dims[l])) for l in range(len(dims) - 1)]
    b = [g.normal(0, scale, size=dims[l + 1]) for l in range(len(dims) - 1)]
    return I.FNet(list(dims), W, b)


def flat(net):
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in zip(net.W, net.b)])


def unflat(dims, theta):
    W, b, t = [], [], 0
    for l in range(len(dims) - 1):
        nw = dims[l + 1] * dims[l]
        W.append(theta[t:t + nw].reshape(dims[l + 1], dims[l]).copy())
        t += nw
        b.append(theta[t:t + dims[l + 1]].copy())
        t += dims[l + 1]
    return I.FNet(list(dims), W, b)


@pytest.mark.parametrize("dims,seed", [([10, 7, 4], 1), ([8, 6, 5, 3], 2)])
def test_gradient_matches_central_differences(orc, dims, seed):
    g = I.rng(seed)
    net = f64net(dims, g)
    imgs = g.integers(0, 256, size=(5, dims[0])).astype(np.uint8)
    labs = g.integers(0, dims[-1], size=5).astype(np.int32)
    _, grad = orc.f64_loss_grad(net, imgs, labs)
    theta = flat(net)
    assert grad.shape == theta.shape
    h = 1e-6
    fd = np.empty_like(theta)
    for t in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[t] += h
        tm[t] -= h
        fd[t] = (orc.f64_loss_grad(unflat(dims, tp), imgs, labs)[0] -
                 orc.f64_loss_grad(unflat(dims, tm), imgs, labs)[0]) / (2 * h)
    assert np.max(np.abs(grad - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))
    assert np.max(np.abs(fd)) > 1e-3


def test_zero_weights_closed_form(orc):
    dims = [6, 5, 4]
    net = I.FNet(dims, [np.zeros((5, 6)), np.zeros((4, 5))], [np.zeros(5), np.zeros(4)])
    g = I.rng(3)
    imgs = g.integers(0, 256, size=(8, 6)).astype(np.uint8)
    labs = np.array([0, 1, 2, 3, 0, 0, 1, 3], np.int32)
    loss, grad = orc.f64_loss_grad(net, imgs, labs)
    assert loss == pytest.approx(np.log(4.0), abs=1e-15)
    onehot = np.eye(4)[labs]
    gb2 = grad[-4:]
    assert np.allclose(gb2, (0.25 - onehot).mean(axis=0), atol=1e-15)
    # hidden units are sigmoid(0) = 1/2: dL/dW2 = gb2 outer 1/2
    assert np.allclose(grad[30 + 5:30 + 5 + 20].reshape(4, 5), np.outer(gb2, np.full(5, 0.5)), atol=1e-15)
    # zero W2 stops the gradient into layer 1
    assert np.all(grad[:35] == 0.0)


def test_single_layer_is_logistic_regression(orc):
    from sklearn.metrics import log_loss
    g = I.rng(4)
    dims = [9, 3]
    net = f64net(dims, g)
    imgs = g.integers(0, 256, size=(20, 9)).astype(np.uint8)
    labs = g.integers(0, 3, size=20).astype(np.int32)
    loss, grad = orc.f64_loss_grad(net, imgs, labs)
    X = imgs / 256.0
    p = softmax(X @ net.W[0].T + net.b[0], axis=1)
    assert loss == pytest.approx(log_loss(labs, p, labels=[0, 1, 2]), rel=1e-12)
    r = (p - np.eye(3)[labs]) / 20.0
    assert np.allclose(grad[:27].reshape(3, 9), r.T @ X, atol=1e-13)
    assert np.allclose(grad[27:], r.sum(axis=0), atol=1e-13)


def test_constant_hidden_layer(orc):
    from sklearn.metrics import log_loss
    g = I.rng(6)
    dims = [7, 4, 3]
    net = f64net(dims, g)
    net.W[0][:] = 0.0
    imgs = g.integers(0, 256, size=(10, 7)).astype(np.uint8)
    labs = g.integers(0, 3, size=10).astype(np.int32)
    loss, _ = orc.f64_loss_grad(net, imgs, labs)
    z = net.W[1] @ expit(net.b[0]) + net.b[1]
    p = np.repeat(softmax(z)[None, :], 10, axis=0)
    assert loss == pytest.approx(log_loss(labs, p, labels=[0, 1, 2]), rel=1e-12)


def test_invariants(orc):
    g = I.rng(8)
    dims = [12, 8, 6, 5]
    net = f64net(dims, g)
    imgs = g.integers(0, 256, size=(7, 12)).astype(np.uint8)
    labs = g.integers(0, 5, size=7).astype(np.int32)
    loss, grad = orc.f64_loss_grad(net, imgs, labs)
    assert abs(grad[-5:].sum()) < 1e-15
    shifted = I.FNet(dims, net.W, net.b[:-1] + [net.b[-1] + 3.25])
    assert orc.f64_loss_grad(shifted, imgs, labs)[0] == pytest.approx(loss, rel=1e-12)
    with pytest.raises(Exception):
        orc.f64_loss_grad(net, imgs, np.array([0, 1, 2, 3, 4, 5, 0], np.int32))


def test_adam_first_step_and_descent(orc):
    g = I.rng(9)
    dims = [10, 6, 3]
    net = f64net(dims, g)
    imgs = g.integers(0, 256, size=(12, 10)).astype(np.uint8)
    labs = g.integers(0, 3, size=12).astype(np.int32)
    _, grad = orc.f64_loss_grad(net, imgs, labs)
    W, b, losses = orc.f64_fit(net, imgs, labs, [np.arange(12)], batch=12, lr=1e-3, eps=1e-12)
    step = flat(I.FNet(dims, W, b)) - flat(net)
    nz = np.abs(grad) > 1e-9
    assert np.allclose(step[nz], -1e-3 * np.sign(grad[nz]), rtol=1e-6, atol=0)
    assert losses[0] == pytest.approx(orc.f64_loss_grad(net, imgs, labs)[0], rel=1e-12)
    # a linearly separable set: two prototypes, labels by prototype
    proto = g.integers(0, 2, size=(2, 10)) * 255
    lab2 = g.integers(0, 2, size=40).astype(np.int32)
    img2 = proto[lab2].astype(np.uint8)
    net2 = f64net([10, 6, 2], g, scale=0.1)
    order = np.stack([g.permutation(40) for _ in range(30)])
    W2, b2, l2 = orc.f64_fit(net2, img2, lab2, order, batch=8, lr=3e-2)
    assert l2[-1] < 0.1 * l2[0]
