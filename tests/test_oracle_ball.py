"""Pins of the oracle's L2-ball domain (the restriction R of Sec. III-C,
Eq. (9), with the Euclidean distance of Eq. (7) on pixel values): the
images x' in {0..255}^n with |x' - x|^2 <= r2, level k = support size.

  - published lattice-point counts of discs and balls (OEIS A000328 and
    A000605) for interior images;
  - brute force over every image near x, on tiny nets, with an independent
    rank encoder (itertools subsets, the offset-to-digit map of the header);
  - at level 1 the ball equals the box domain with D = {-rd..-1, 1..rd}, at
    level 2 it is that box filtered by the squared distance (interior x);
  - an empty ball and images on the [0, 255] boundary."""
import itertools
import os

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def published_counts():
    out = {}
    for line in open(os.path.join(HERE, "golden", "lattice_ball_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t) for t in line.split()]
        out[v[0]] = v[1:]
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_lattice_counts_match_published(orc, d):
    counts = published_counts()[d]
    net = I.random_qnet(I.rng(d), [d, 8, 3], shift=4)
    x = np.full(d, 128, np.uint8)
    for r, want in enumerate(counts):
        res = orc.q8_ball_check(net, x, r * r, k_min=0, k_max=d)
        assert int(res["points"].sum()) == want, (d, r)


def offset_digit(e, rd):
    return e + rd if e < 0 else e + rd - 1


def brute_force(orc, net, x, r2):
    """Every image within r2 of x, by support size: points, records, ties."""
    n = len(x)
    rd = int(np.floor(np.sqrt(r2)))
    rd = min(rd, 255)
    m = 2 * rd
    _, clean = orc.q8_forward(net, x)
    subsets = {k: {s: i for i, s in enumerate(itertools.combinations(range(n), k))} for k in range(n + 1)}
    ranges = [range(max(0, int(v) - rd), min(255, int(v) + rd) + 1) for v in x]
    points = np.zeros(n + 1, np.int64)
    ties = np.zeros(n + 1, np.int64)
    recs = set()
    nc = net.dims[-1]
    for xp in itertools.product(*ranges):
        e = np.array(xp, np.int64) - x.astype(np.int64)
        if int((e * e).sum()) > r2:
            continue
        S = tuple(int(p) for p in np.nonzero(e)[0])
        k = len(S)
        points[k] += 1
        pot, lab = orc.q8_forward(net, np.array(xp, np.uint8))
        z = pot[-nc:]
        if np.sum(z == z.max()) > 1:
            ties[k] += 1
        if k and lab != clean:
            rank = subsets[k][S]
            for p in S:
                rank = rank * m + offset_digit(int(e[p]), rd)
            recs.add((k, rank, lab))
    return points, ties, recs, m


@pytest.mark.parametrize("seed,x,r2,unsafe", [
    (41, [128, 128, 128], 20, True),
    (112, [0, 128, 255], 30, True),     # offsets that leave [0, 255] are not images
    (27, [1, 254, 3], 12, True),
    (4, [200, 7, 90], 2, False),
])
def test_brute_force_tiny_nets(orc, seed, x, r2, unsafe):
    g = I.rng(500 + seed)
    net = I.random_qnet(g, [3, 12, 4], shift=3, wmax=40, bmax=200)
    x = np.array(x, np.uint8)
    pts, ties, recs, m = brute_force(orc, net, x, r2)
    res = orc.q8_ball_check(net, x, r2, k_min=0, k_max=3)
    assert res["m"] == m
    assert list(res["points"]) == list(pts)
    assert list(res["ties"][1:]) == list(ties[1:])
    got = set(zip(res["cex_k"].tolist(), res["cex_rank"].tolist(), res["cex_label"].tolist()))
    assert got == recs and (len(recs) > 0) == unsafe
    assert sum(res["cex"]) == len(recs)
    # records come out sorted by (k, rank)
    key = list(zip(res["cex_k"].tolist(), res["cex_rank"].tolist()))
    assert key == sorted(key)


def test_level1_is_the_box_and_level2_its_ball_part(orc):
    g = I.rng(5)
    net = I.random_qnet(g, [10, 32, 6], shift=5, wmax=30, bmax=300)
    x = g.integers(40, 215, size=10, endpoint=True).astype(np.uint8)   # interior: no offset leaves [0, 255]
    r2 = 40                                                            # rd = 6
    rd = orc.ball_digits(r2)
    assert rd == 6
    D = np.array(list(range(-rd, 0)) + list(range(1, rd + 1)), np.int16)
    ball = orc.q8_ball_check(net, x, r2, k_min=1, k_max=2)
    box = orc.q8_check(net, x, D, k_min=1, k_max=2)
    assert box["cex_total"] > 0
    # level 1: identical
    b1 = box["cex_k"] == 1
    a1 = ball["cex_k"] == 1
    assert ball["points"][0] == box["points"][0] == 10 * 12
    assert np.array_equal(ball["cex_rank"][a1], box["cex_rank"][b1])
    assert np.array_equal(ball["cex_label"][a1], box["cex_label"][b1])
    # level 2: the box records whose two offsets lie inside the ball
    keep = []
    for k, r, lab in zip(box["cex_k"], box["cex_rank"], box["cex_label"]):
        if k != 2:
            continue
        pix, dig = orc.decode(10, len(D), 2, int(r))
        if int(D[dig[0]]) ** 2 + int(D[dig[1]]) ** 2 <= r2:
            keep.append((int(r), int(lab)))
    a2 = ball["cex_k"] == 2
    assert keep == list(zip(ball["cex_rank"][a2].tolist(), ball["cex_label"][a2].tolist()))
    pairs = sum(1 for a in D for b in D if int(a) ** 2 + int(b) ** 2 <= r2)
    assert ball["points"][1] == 45 * pairs


def test_empty_ball(orc):
    net = I.random_qnet(I.rng(3), [5, 8, 3], shift=4)
    x = np.arange(5, dtype=np.uint8) * 40
    res = orc.q8_ball_check(net, x, 0, k_min=0, k_max=2)
    assert list(res["points"]) == [1, 0, 0] and res["cex_total"] == 0 and res["m"] == 0
