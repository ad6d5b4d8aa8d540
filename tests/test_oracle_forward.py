"""Pins of the oracle's forward passes against numpy's own matmul (a library
routine, not a retyped loop) on seeded random networks."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I


def numpy_q8(net, x):
    a = x.astype(np.int64)
    pots = []
    for l, (W, b) in enumerate(zip(net.W, net.b)):
        u = W.astype(np.int64) @ a + b.astype(np.int64)
        pots.append(u)
        if l < net.n_layers - 1:
            a = np.clip(np.floor_divide(u, 2 ** net.shift[l]), 0, 127)
        else:
            a = u
    return np.concatenate(pots), int(np.argmax(a))


@pytest.mark.parametrize("dims,shift", [([35, 16, 5], 7), ([64, 32, 10], 5), ([20, 9, 7, 3], 3),
                                        ([784, 256, 256, 10], 7), ([9, 4, 4, 4, 2], 0)])
def test_q8_forward_matches_numpy(orc, dims, shift):
    g = I.rng(11)
    net = I.random_qnet(g, dims, shift=shift)
    for _ in range(20):
        x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
        pot, lab = orc.q8_forward(net, x)
        ref, rlab = numpy_q8(net, x)
        assert np.array_equal(pot, ref)
        assert lab == rlab


def test_q8_forward_lowest_index_tie(orc):
    # two equal logits: the label is the lower index
    net = I.QNet([2, 2], [np.array([[1, 0], [0, 1]], np.int8)], [np.zeros(2, np.int32)], [])
    _, lab = orc.q8_forward(net, np.array([7, 7], np.uint8))
    assert lab == 0
    _, lab = orc.q8_forward(net, np.array([7, 8], np.uint8))
    assert lab == 1


def test_q8_forward_floor_shift_negative(orc):
    # floor(-1 / 2) = -1 -> clamped to 0; floor(255/2) = 127; floor(3/2) = 1
    net = I.QNet([1, 1, 1], [np.array([[1]], np.int8), np.array([[1]], np.int8)],
                 [np.array([-4], np.int32), np.zeros(1, np.int32)], [1])
    pot, _ = orc.q8_forward(net, np.array([3], np.uint8))
    assert list(pot) == [-1, 0]
    pot, _ = orc.q8_forward(net, np.array([7], np.uint8))
    assert list(pot) == [3, 1]


def test_q8_forward_range_error(orc):
    net = I.QNet([2, 1], [np.array([[127, 127]], np.int8)], [np.array([2**31 - 10], np.int32)], [])
    with pytest.raises(orc.OracleError):
        orc.q8_forward(net, np.array([255, 255], np.uint8))


def test_f64_forward_matches_numpy(orc):
    g = I.rng(12)
    q = I.random_qnet(g, [30, 12, 8, 4])
    net = I.fnet_from_qnet(q)
    for _ in range(10):
        x = g.integers(0, 255, size=30, endpoint=True).astype(np.uint8)
        pot, lab, mg = orc.f64_forward(net, x)
        a = x.astype(np.float64) / 256.0
        ref = []
        for l, (W, b) in enumerate(zip(net.W, net.b)):
            u = W.astype(np.float64) @ a + b.astype(np.float64)
            ref.append(u)
            a = 1.0 / (1.0 + np.exp(-u)) if l < 2 else u
        ref = np.concatenate(ref)
        np.testing.assert_allclose(pot, ref, rtol=1e-12, atol=1e-12)
        assert lab == int(np.argmax(a))
        s = np.sort(a)
        assert abs(mg - (s[-1] - s[-2])) < 1e-12


def test_euclid_worked_example(orc):
    # Sec. III-C: the distance of the two 5x5 binary glyphs "A" and "O" is
    # printed as 2.449, i.e. sqrt(6): six pixels differ by one unit.
    g = I.rng(3)
    p = (g.random(25) < 0.5).astype(np.float64)
    q = p.copy()
    flip = g.choice(25, 6, replace=False)
    q[flip] = 1.0 - q[flip]
    assert abs(orc.euclid(p, q) - 2.449) < 5e-4
    assert orc.euclid(p, p) == 0.0


def numpy_f64(net, X):
    """Logits of images X [B][n] by numpy's float64 matmul and exp."""
    a = X.astype(np.float64) / 256.0
    for l, (W, b) in enumerate(zip(net.W, net.b)):
        u = a @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        a = 1.0 / (1.0 + np.exp(-u)) if l < len(net.W) - 1 else u
    return a


@pytest.mark.parametrize("dims", [[6, 8, 4], [7, 5, 6, 3], [6, 9, 4, 4, 2]])
def test_f64_eval_points_matches_numpy(orc, dims):
    """orc_f64_eval_points: every point of levels 0..3, decoded here by
    itertools' lexicographic order and applied with numpy, gives numpy's
    float64 logits, the lowest-index argmax and the top-2 margin."""
    import itertools
    g = I.rng(23)
    net = I.fnet_from_qnet(I.random_qnet(g, dims, shift=7))
    n = dims[0]
    x = g.integers(0, 255, size=n, endpoint=True).astype(np.uint8)
    D = np.array([-200, -5, 0, 60], np.int16)
    ks, ranks, imgs = [], [], []
    for k in range(0, 4):
        rank = 0
        for S in itertools.combinations(range(n), k):
            for dig in itertools.product(range(len(D)), repeat=k):
                xp = x.astype(np.int64).copy()
                for p, i in zip(S, dig):
                    xp[p] = min(max(int(x[p]) + int(D[i]), 0), 255)
                ks.append(k); ranks.append(rank); imgs.append(xp)
                rank += 1
    labels, logits, margins = orc.f64_eval_points(net, x, D, ks, ranks)
    ref = numpy_f64(net, np.array(imgs))
    assert np.allclose(logits, ref, rtol=1e-12, atol=1e-12)
    assert np.array_equal(labels, np.argmax(ref, axis=1))
    srt = np.sort(ref, axis=1)
    assert np.allclose(margins, srt[:, -1] - srt[:, -2], rtol=1e-9, atol=1e-12)


def test_f64_eval_points_closed_form(orc):
    """The O3 net (identity first layer, logits +-(a0 - a1) with
    a = sigmoid(x / 256)): margin 2 |a0 - a1|, class 0 iff x0' >= x1'."""
    net = I.FNet([2, 2, 2], [np.eye(2), np.array([[1.0, -1.0], [-1.0, 1.0]])], [np.zeros(2), np.zeros(2)])
    x = np.array([100, 90], np.uint8)
    D = np.arange(-16, 17, dtype=np.int16)
    ranks = np.arange(33 * 33)
    labels, logits, margins = orc.f64_eval_points(net, x, D, np.full(ranks.size, 2), ranks)
    d0, d1 = np.divmod(ranks, 33)
    x0, x1 = 100 + D[d0].astype(np.int64), 90 + D[d1].astype(np.int64)
    sig = lambda v: 1.0 / (1.0 + np.exp(-v / 256.0))
    assert np.array_equal(labels, np.where(x0 >= x1, 0, 1))
    assert np.allclose(margins, 2 * np.abs(sig(x0) - sig(x1)), rtol=1e-12, atol=1e-15)
    assert np.allclose(logits[:, 0], sig(x0) - sig(x1), rtol=1e-12, atol=1e-15)
