"""Pins of the oracle's exhaustive check: closed forms on 2-2-2 nets, brute
force over tiny nets, rank/decode against itertools' lexicographic order,
and the invariants of the method."""
import itertools

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

D33 = np.arange(-16, 17, dtype=np.int16)


def diff_net(w1=1, shift=0):
    """2-2-2 net: a = clamp(floor(w1*x / 2^shift), 0, 127), logits (a0-a1, a1-a0)."""
    return I.QNet([2, 2, 2], [np.array([[w1, 0], [0, w1]], np.int8), np.array([[1, -1], [-1, 1]], np.int8)],
                  [np.zeros(2, np.int32), np.zeros(2, np.int32)], [shift])


@pytest.mark.parametrize("x,w1,shift,deltas,expect_cex,expect_ties,clean", [
    # P1: label 0 while x0' >= x1'.  k=1: d0 <= -11 (6) or d1 >= 11 (6);
    # k=2: d1 - d0 >= 11, sum_{s=1}^{22} s = 253; ties: 2 at k=1, 23 at k=2.
    ((100, 90), 1, 0, D33, [12, 253], [2, 23], 0),
    # P2: x = (5, 10), label 1; clamping at 0 collapses negative deltas on pixel 0.
    ((5, 10), 1, 0, D33, [24, 462], None, 1),
    # P3: W1 = 64 I, shift 7, so a = floor(x/2): floor requantisation.
    ((100, 90), 64, 7, D33, [11, 242], None, 0),
    # P4a: every activation saturates at 127 -> permanent tie -> no counterexample.
    ((250, 240), 1, 0, D33, [0, 0], [66, 1089], 0),
    # P4b: sparse delta set.
    ((100, 90), 1, 0, np.array([-32, -16, -8, 8, 16, 32], np.int16), [4, 13], None, 0),
])
def test_closed_form(orc, x, w1, shift, deltas, expect_cex, expect_ties, clean):
    r = orc.q8_check(diff_net(w1, shift), np.array(x, np.uint8), deltas, 1, 2)
    assert r["clean_label"] == clean
    assert list(r["cex"]) == expect_cex
    if expect_ties is not None:
        assert list(r["ties"]) == expect_ties
    m = len(deltas)
    assert list(r["points"]) == [2 * m, m * m]


def test_closed_form_by_counting(orc):
    # P2 and P3 counts re-derived here by counting the closed-form condition
    # over the deltas (label 0 iff a0 >= a1 with a = clamp(floor(x/2^s)...)).
    def lab(a0, a1):
        return 0 if a0 >= a1 else 1
    for x, w1, sh in [((5, 10), 1, 0), ((100, 90), 64, 7), ((100, 90), 1, 0), ((0, 255), 1, 0)]:
        act = lambda v: min(max((w1 * v) >> sh, 0), 127)
        cl = lab(act(x[0]), act(x[1]))
        k1 = sum(lab(act(min(max(x[0] + d, 0), 255)), act(x[1])) != cl for d in D33) + \
             sum(lab(act(x[0]), act(min(max(x[1] + d, 0), 255))) != cl for d in D33)
        k2 = sum(lab(act(min(max(x[0] + d0, 0), 255)), act(min(max(x[1] + d1, 0), 255))) != cl
                 for d0 in D33 for d1 in D33)
        r = orc.q8_check(diff_net(w1, sh), np.array(x, np.uint8), D33, 1, 2)
        assert list(r["cex"]) == [k1, k2]


def test_float_closed_form(orc):
    # O3 pin: the P1 net in float with sigmoid hidden units: sigmoid is
    # monotone, so the decision is x0' >= x1' and the counts are P1's; the
    # exact ties have margin 0 and are flagged.
    q = diff_net()
    f = I.FNet([2, 2, 2], [np.eye(2), np.array([[1.0, -1.0], [-1.0, 1.0]])], [np.zeros(2), np.zeros(2)])
    r = orc.f64_check(f, np.array([100, 90], np.uint8), D33, 1, 2, tie_rel=1e-12)
    assert list(r["cex"]) == [12, 253]
    assert list(r["ties"]) == [2, 23]
    assert np.all(r["tie_margin"] == 0.0)
    rq = orc.q8_check(q, np.array([100, 90], np.uint8), D33, 1, 2)
    assert np.array_equal(r["cex_rank"], rq["cex_rank"])


def enumerate_points(n, D, k):
    """Independent enumeration: itertools yields subsets and delta tuples in
    lexicographic order, so the position in this nested loop is the rank."""
    for S in itertools.combinations(range(n), k):
        for dig in itertools.product(range(len(D)), repeat=k):
            yield S, dig


def apply(x, D, S, dig):
    xp = x.astype(np.int64).copy()
    for p, i in zip(S, dig):
        xp[p] = min(max(int(x[p]) + int(D[i]), 0), 255)
    return xp.astype(np.uint8)


@pytest.mark.parametrize("n,m,k", [(5, 3, 0), (5, 3, 1), (5, 3, 2), (6, 2, 3), (6, 2, 6), (7, 4, 3), (4, 5, 4)])
def test_decode_and_count_match_itertools(orc, n, m, k):
    D = np.arange(m, dtype=np.int16)
    pts = list(enumerate_points(n, D, k))
    assert orc.points(n, m, k) == len(pts)
    for rank, (S, dig) in enumerate(pts):
        pix, dd = orc.decode(n, m, k, rank)
        assert tuple(pix) == S and tuple(dd) == dig


@pytest.mark.parametrize("seed,dims", [(1, [4, 3, 3]), (2, [5, 4, 3]), (3, [6, 3, 2, 3]), (4, [5, 6, 4])])
def test_bruteforce_small(orc, seed, dims):
    g = I.rng(seed)
    net = I.random_qnet(g, dims, shift=3, wmax=20, bmax=200)
    n = dims[0]
    x = g.integers(0, 255, size=n, endpoint=True).astype(np.uint8)
    D = np.array([-40, -9, 0, 7, 33], np.int16)
    _, clean = orc.q8_forward(net, x)
    r = orc.q8_check(net, x, D, 0, n)
    # (a) every level: the (k, rank, label) list equals the itertools scan
    exp_k, exp_r, exp_l = [], [], []
    for k in range(0, n + 1):
        for rank, (S, dig) in enumerate(enumerate_points(n, D, k)):
            _, lab = orc.q8_forward(net, apply(x, D, S, dig))
            if lab != clean:
                exp_k.append(k); exp_r.append(rank); exp_l.append(lab)
    assert list(r["cex_k"]) == exp_k and list(r["cex_rank"]) == exp_r and list(r["cex_label"]) == exp_l
    # (b) "fully unwound": with 0 in D the union over all levels of the
    # misclassified images equals the misclassified images of the whole box D^n
    found = set()
    for k, rank in zip(r["cex_k"], r["cex_rank"]):
        pix, dd = orc.decode(n, len(D), int(k), int(rank))
        found.add(apply(x, D, tuple(pix), tuple(dd)).tobytes())
    box = set()
    for dig in itertools.product(range(len(D)), repeat=n):
        xp = apply(x, D, tuple(range(n)), dig)
        if orc.q8_forward(net, xp)[1] != clean:
            box.add(xp.tobytes())
    assert found == box


def test_invariants_glyph35(orc):
    w = I.workload_glyph35()
    x = w.images[3]
    r = orc.q8_check(w.net, x, w.deltas, 0, 2)
    assert list(r["levels"]) == [0, 1, 2]
    assert list(r["points"]) == [1, 35 * 33, 595 * 33 * 33]
    # k = 0 is the clean image: never a counterexample
    assert r["cex"][0] == 0
    # replay: every counterexample decodes to an image with the reported label
    labels = orc.q8_eval_points(w.net, x, w.deltas, r["cex_k"], r["cex_rank"])
    assert np.array_equal(labels, r["cex_label"])
    assert np.all(labels != r["clean_label"])
    # zero perturbation (0 in D) reproduces the clean label
    zi = int(np.where(w.deltas == 0)[0][0])
    for k in (1, 2):
        ranks = []
        for S_rank in range(0, 35 if k == 1 else 595, 7):
            ranks.append(S_rank * 33 ** k + sum(zi * 33 ** (k - 1 - j) for j in range(k)))
        lab = orc.q8_eval_points(w.net, x, w.deltas, [k] * len(ranks), ranks)
        assert np.all(lab == r["clean_label"])
    # containment: with 0 in D the misclassified images at k are also found at k+1
    imgs = {1: set(), 2: set()}
    for k, rank in zip(r["cex_k"], r["cex_rank"]):
        pix, dd = orc.decode(35, 33, int(k), int(rank))
        imgs[int(k)].add(apply(x, w.deltas, tuple(pix), tuple(dd)).tobytes())
    assert imgs[1] <= imgs[2]


def test_stop_at_first_and_capacity(orc):
    r = orc.q8_check(diff_net(), np.array([100, 90], np.uint8), D33, 1, 2, stop_at_first=True)
    assert r["first_unsafe_k"] == 1 and list(r["levels"]) == [1]
    r = orc.q8_check(diff_net(), np.array([100, 90], np.uint8), D33, 1, 2, cap=5)
    assert r["cex_total"] == 265 and len(r["cex_rank"]) == 5
    full = orc.q8_check(diff_net(), np.array([100, 90], np.uint8), D33, 1, 2)
    assert np.array_equal(full["cex_rank"][:5], r["cex_rank"])


def test_k_step(orc):
    w = I.workload_glyph35()
    r = orc.q8_check(w.net, w.images[0], w.deltas[::4], 1, 3, k_step=2)
    assert list(r["levels"]) == [1, 3]
    assert list(r["points"]) == [35 * 9, 6545 * 9 ** 3]
