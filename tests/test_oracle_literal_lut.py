"""Pins of the oracle's threshold literal (Sec. III-C: the image is
misclassified when the desired class's output falls below the reference
value V and another class's rises above it) and of its table sigmoid (the
paper's CUDA code took the sigmoid from a table, Sec. IV-D).

  - the table sigmoid: its knots are the FP32-rounded sigmoid, it is linear
    between knots, saturates outside [-8, 8], is nondecreasing, and stays
    within the linear-interpolation error bound h^2/8 max|sigma''| of the
    sigmoid (h = 1/16);
  - the literal: brute force over every point of small domains with an
    independent numpy forward (integer and double), the decision written as
    its definition, against the oracle's records, counts and ties;
  - the table-sigmoid check: the same brute force with the pinned table
    function in place of the sigmoid."""
import itertools
import math

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I


def sigmoid(u):
    return 1.0 / (1.0 + math.exp(-u))


def test_table_sigmoid(orc):
    knots = [-8.0 + i / 16.0 for i in range(257)]
    for u in knots:
        assert orc.lut_sigmoid(u) == float(np.float32(sigmoid(u)))
    # linear between knots
    for i in range(0, 256, 7):
        a, c = orc.lut_sigmoid(knots[i]), orc.lut_sigmoid(knots[i + 1])
        for f in (0.25, 0.5, 0.75):
            assert abs(orc.lut_sigmoid(knots[i] + f / 16.0) - (a + f * (c - a))) < 1e-15
    # saturation and monotonicity
    assert orc.lut_sigmoid(-50.0) == orc.lut_sigmoid(-8.0) and orc.lut_sigmoid(40.0) == orc.lut_sigmoid(8.0)
    grid = np.linspace(-10, 10, 20001)
    vals = np.array([orc.lut_sigmoid(u) for u in grid])
    assert np.all(np.diff(vals) >= 0)
    # interpolation error: h^2 / 8 * max|sigma''| (= 1 / (6 sqrt 3)) plus FP32 rounding of the knots
    inside = np.abs(grid) <= 8
    err = np.abs(vals[inside] - 1.0 / (1.0 + np.exp(-grid[inside])))
    bound = (1.0 / 16.0) ** 2 / 8.0 / (6.0 * math.sqrt(3.0)) + 6e-8
    assert err.max() <= bound and err.max() > 0.5 * bound


def int_forward(net, x):
    a = x.astype(np.int64)
    for l in range(len(net.W)):
        u = net.W[l].astype(np.int64) @ a + net.b[l].astype(np.int64)
        if l < len(net.W) - 1:
            a = np.clip(np.floor_divide(u, 1 << net.shift[l]), 0, 127)
        else:
            a = u
    return a


def float_forward(net, x, act):
    a = x.astype(np.float64) / 256.0
    for l in range(len(net.W)):
        u = net.W[l].astype(np.float64) @ a + net.b[l].astype(np.float64)
        a = np.array([act(v) for v in u]) if l < len(net.W) - 1 else u
    return a


def domain(n, D, kmax):
    """(k, rank, pixels, deltas) of every point of levels 1..kmax, rank order."""
    m = len(D)
    for k in range(1, kmax + 1):
        for s_rank, S in enumerate(itertools.combinations(range(n), k)):
            for d_rank, ds in enumerate(itertools.product(range(m), repeat=k)):
                yield k, s_rank * m ** k + d_rank, S, ds


def apply(x, D, S, ds):
    y = x.astype(np.int64).copy()
    for p, d in zip(S, ds):
        y[p] = min(255, max(0, y[p] + int(D[d])))
    return y.astype(np.uint8)


def literal(z, Dc, V):
    other = max(z[i] for i in range(len(z)) if i != Dc)
    return z[Dc] < V and other > V, (z[Dc] == V) or (other == V)


@pytest.mark.parametrize("seed", [601, 607])
def test_integer_literal_brute_force(orc, seed):
    g = I.rng(seed)
    net = I.random_qnet(g, [6, 8, 3], shift=4, wmax=30, bmax=200)
    x = g.integers(0, 255, size=6, endpoint=True).astype(np.uint8)
    D = np.array([-90, -40, 40, 90], np.int16)
    z0 = int_forward(net, x)
    Dc = int(np.argmax(z0))
    V = int(np.sort(z0)[-2] + (z0[Dc] - np.sort(z0)[-2]) // 2)     # between the top two clean logits
    recs, ties = set(), [0, 0]
    for k, rank, S, ds in domain(6, D, 2):
        z = int_forward(net, apply(x, D, S, ds))
        v, t = literal(list(z), Dc, V)
        ties[k - 1] += t
        if v:
            recs.add((k, rank, int(np.argmax(z))))
    r = orc.q8_check_literal(net, x, D, V, 1, 2)
    assert r["clean_label"] == Dc
    assert set(zip(r["cex_k"].tolist(), r["cex_rank"].tolist(), r["cex_label"].tolist())) == recs
    assert list(r["ties"]) == ties and len(recs) > 0


@pytest.mark.parametrize("lut,seed", [(False, 658), (True, 658), (True, 673)])
def test_float_literal_and_table_brute_force(orc, lut, seed):
    g = I.rng(seed)
    net = I.fnet_from_qnet(I.random_qnet(g, [6, 8, 4, 3], shift=4, wmax=60, bmax=4000))
    x = g.integers(0, 255, size=6, endpoint=True).astype(np.uint8)
    D = np.array([-120, -50, 50, 120], np.int16)
    act = orc.lut_sigmoid if lut else sigmoid
    z0 = float_forward(net, x, act)
    Dc = int(np.argmax(z0))
    V = float((np.sort(z0)[-1] + np.sort(z0)[-2]) / 2)
    recs = set()
    for k, rank, S, ds in domain(6, D, 2):
        z = float_forward(net, apply(x, D, S, ds), act)
        if literal(list(z), Dc, V)[0]:
            recs.add((k, rank))
    r = orc.f64_check(net, x, D, 1, 2, tie_rel=0.0, lut=lut, literal_v=V)
    assert set(zip(r["cex_k"].tolist(), r["cex_rank"].tolist())) == recs and len(recs) > 0
    # the plain property with the table sigmoid: label changes
    if lut:
        lab = set()
        for k, rank, S, ds in domain(6, D, 2):
            z = float_forward(net, apply(x, D, S, ds), act)
            if int(np.argmax(z)) != Dc:
                lab.add((k, rank))
        r2 = orc.f64_check(net, x, D, 1, 2, tie_rel=0.0, lut=True)
        assert set(zip(r2["cex_k"].tolist(), r2["cex_rank"].tolist())) == lab
