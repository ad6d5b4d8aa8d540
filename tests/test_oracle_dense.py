"""Pins of the block-matrix form of the oracle's integer check (oracle/dense.py):
the closed forms of the 2-2-2 nets, the itertools brute force over tiny nets,
and record-for-record agreement with the C oracle on nets that take both the
float32 and the float64 product paths."""
import itertools

import numpy as np
import pytest

from oracle import dense
from paper_1907_12933_amd import inputs as I

from test_oracle_check import D33, diff_net, enumerate_points, apply


@pytest.mark.parametrize("x,w1,shift,deltas,expect_cex,expect_ties,clean", [
    ((100, 90), 1, 0, D33, [12, 253], [2, 23], 0),
    ((5, 10), 1, 0, D33, [24, 462], None, 1),
    ((100, 90), 64, 7, D33, [11, 242], None, 0),
    ((250, 240), 1, 0, D33, [0, 0], [66, 1089], 0),
    ((100, 90), 1, 0, np.array([-32, -16, -8, 8, 16, 32], np.int16), [4, 13], None, 0),
])
def test_dense_closed_form(x, w1, shift, deltas, expect_cex, expect_ties, clean):
    r = dense.q8_check(diff_net(w1, shift), np.array(x, np.uint8), deltas, 1, 2)
    assert r["clean_label"] == clean
    assert list(r["cex"]) == expect_cex
    if expect_ties is not None:
        assert list(r["ties"]) == expect_ties
    m = len(deltas)
    assert list(r["points"]) == [2 * m, m * m]


@pytest.mark.parametrize("seed,dims", [(1, [4, 3, 3]), (3, [6, 3, 2, 3]), (4, [5, 6, 4])])
def test_dense_bruteforce_small(orc, seed, dims):
    g = I.rng(seed)
    net = I.random_qnet(g, dims, shift=3, wmax=20, bmax=200)
    n = dims[0]
    x = g.integers(0, 255, size=n, endpoint=True).astype(np.uint8)
    D = np.array([-40, -9, 0, 7, 33], np.int16)
    _, clean = orc.q8_forward(net, x)
    r = dense.q8_check(net, x, D, 0, n, block=64)
    exp_k, exp_r, exp_l = [], [], []
    for k in range(0, n + 1):
        for rank, (S, dig) in enumerate(enumerate_points(n, D, k)):
            _, lab = orc.q8_forward(net, apply(x, D, S, dig))
            if lab != clean:
                exp_k.append(k); exp_r.append(rank); exp_l.append(lab)
    assert list(r["cex_k"]) == exp_k and list(r["cex_rank"]) == exp_r and list(r["cex_label"]) == exp_l


@pytest.mark.parametrize("seed,dims,wmax,shift,deltas,kmax", [
    (11, [30, 64, 32, 7], 64, 5, [-48, -16, 16, 48], 2),      # float32 products
    (12, [40, 48, 9], 127, 6, [-64, 64], 3),                 # float32, three levels
    (14, [784, 96, 10], 127, 11, [-64, 64], 2),              # 784 * 127 * 255 >= 2^24: float64
])
def test_dense_matches_c_oracle(orc, seed, dims, wmax, shift, deltas, kmax):
    g = I.rng(seed)
    net = I.random_qnet(g, dims, shift=shift, wmax=wmax, bmax=512)
    if dims[0] == 784:
        # one full-magnitude row: its partial sums reach 784 * 127 * 255 > 2^24
        net.W[0][0, :] = np.where(net.W[0][0, :] >= 0, 127, -127)
    x = I.blob_images(g, 1)[0] if dims[0] == 784 else g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    D = np.array(deltas, np.int16)
    a = dense.q8_check(net, x, D, 1, kmax)
    b = orc.q8_check(net, x, D, 1, kmax)
    assert a["clean_label"] == b["clean_label"]
    assert list(a["cex"]) == list(b["cex"]) and list(a["ties"]) == list(b["ties"])
    assert np.array_equal(a["cex_k"], b["cex_k"]) and np.array_equal(a["cex_rank"], b["cex_rank"])
    assert np.array_equal(a["cex_label"], b["cex_label"])
    # the case exercises both decisions
    assert a["cex_total"] > 0 and a["cex_total"] < sum(a["points"])
    want = np.float64 if dims[0] == 784 else np.float32
    assert dense._Net(net).dt[0] == want


@pytest.mark.parametrize("dims,shift", [([35, 16, 5], 7), ([60, 130, 70, 40, 7], [5, 4, 3]),
                                        ([784, 1024, 1024, 1024, 10], 7)])
def test_dense_potentials_match_c_oracle(orc, dims, shift):
    """The block-matrix potentials (every layer, Eq. (1)) equal the C
    oracle's per-image integer forward."""
    from oracle import dense
    g = I.rng(77)
    net = I.random_qnet(g, dims, shift=shift)
    X = g.integers(0, 255, size=(9, dims[0]), endpoint=True).astype(np.uint8)
    P = dense.q8_potentials(net, X, block=4)
    assert P.shape == (9, sum(dims[1:]))
    for i in range(9):
        assert np.array_equal(P[i], orc.q8_forward(net, X[i])[0])
