"""Pins of the oracle's coverage criteria: the paper's two worked examples
(Table I and Table II, read from tests/golden), plus invariants."""
import os

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def table1():
    rows = read_rows("table1_potentials.txt")
    return {r[0]: np.array([int(v) for v in r[2:]], np.int64) for r in rows}


def bit(bits, t):
    return (int(bits[t // 64]) >> (t % 64)) & 1


def test_table1_pairs_named_by_the_paper(orc):
    pots = table1()
    widths = [3, 2, 1]
    offs = [0, 6]                       # block offsets: 3x2 then 2x1
    for crit, pair, npairs, nneur, named in read_rows("table1_coverage.txt"):
        a, b = pair.split(",")
        r = orc.coverage(widths, pots[a][None], pots[b][None], crit, dist_sq_min=10000,
                         ratio_num=3, ratio_den=2)
        assert r["covered_pairs"] == int(npairs), (crit, pair)
        assert r["covered_neurons"] == int(nneur), (crit, pair)
        assert r["total_pairs"] == 8 and r["total_neurons"] == 6
        if named != "-":
            for trip in named.split(";"):
                l, i, j = (int(v) for v in trip.split(","))
                assert bit(r["bits"], offs[l] + i * widths[l + 1] + j), (crit, pair, trip)


def test_table1_symmetry_and_self(orc):
    pots = table1()
    names = list(pots)
    for crit in ("SS", "DS", "SV", "DV"):
        for a in names:
            for b in names:
                r1 = orc.coverage([3, 2, 1], pots[a][None], pots[b][None], crit, 10000)
                r2 = orc.coverage([3, 2, 1], pots[b][None], pots[a][None], crit, 10000)
                assert np.array_equal(r1["bits"], r2["bits"])
                if a == b:
                    assert r1["covered_pairs"] == 0


def test_table1_thresholds(orc):
    # The SV pair (n22, n13) of (Ex2, Ex3) needs a ratio <= 0.353/0.176 = 2.0057;
    # DS of (Ex2, Ex3) needs a distance <= 0.1822 (squared 33200 in x1000 units).
    pots = table1()
    sv = lambda num, den: orc.coverage([3, 2, 1], pots["Ex2"][None], pots["Ex3"][None], "SV",
                                       ratio_num=num, ratio_den=den)["covered_pairs"]
    assert sv(2, 1) == 1 and sv(201, 100) == 0
    ds = lambda t: orc.coverage([3, 2, 1], pots["Ex2"][None], pots["Ex3"][None], "DS",
                                dist_sq_min=t)["covered_pairs"]
    assert ds(33200) == 3 and ds(33201) == 0


def test_table2_sign_sign(orc):
    rows = read_rows("table2_potentials.txt")
    u = np.array([int(r[1]) for r in rows], np.int64)
    v = np.array([int(r[2]) for r in rows], np.int64)
    widths = [5, 4, 5]
    r = orc.coverage(widths, u[None], v[None], "SS", P=0.8)
    # the paper: pairs (n11, n42) and (n42, n53); 3 of 14 neurons; literal false
    assert r["covered_pairs"] == 2
    assert r["covered_neurons"] == 3 and r["total_neurons"] == 14
    assert abs(r["fraction"] - 3 / 14) < 1e-12 and round(100 * r["fraction"]) == 21
    assert r["literal"] is False
    assert bit(r["bits"], 0 * 4 + 3)            # (n11, n42): block 0, i=0, j=3
    assert bit(r["bits"], 20 + 3 * 5 + 4)       # (n42, n53): block 1 at offset 5*4=20, i=3, j=4
    # the literal turns true once P is at most the covered fraction
    assert orc.coverage(widths, u[None], v[None], "SS", P=3 / 14)["literal"] is True
    # other criteria on the same pair: no layer without a sign change, so no
    # distance change and neither DS nor DV pairs
    assert orc.coverage(widths, u[None], v[None], "DS")["covered_pairs"] == 0
    assert orc.coverage(widths, u[None], v[None], "DV")["covered_pairs"] == 0
    # SV: the single condition sign change in layers 1 and 2 pairs with every
    # next-layer neuron whose magnitude ratio is >= 3/2 without a sign change
    sv = orc.coverage(widths, u[None], v[None], "SV")
    assert sv["covered_pairs"] == 3 and sv["covered_neurons"] == 5
    assert orc.coverage(widths, u[None], v[None], "SV", ratio_num=2, ratio_den=1)["covered_pairs"] == 1


def test_coverage_union_over_pairs(orc):
    # covered set of a batch is the union of the per-pair sets
    g = I.rng(9)
    net = I.random_qnet(g, [20, 12, 8, 5], shift=4, wmax=30, bmax=300)
    x1 = g.integers(0, 255, size=(6, 20), endpoint=True).astype(np.uint8)
    x2 = np.stack([I.perturbed_partner(g, x, 6, 40) for x in x1])
    P1 = np.stack([orc.q8_forward(net, x)[0] for x in x1])
    P2 = np.stack([orc.q8_forward(net, x)[0] for x in x2])
    for crit in ("SS", "DS", "SV", "DV"):
        whole = orc.coverage([12, 8, 5], P1, P2, crit)["bits"]
        acc = np.zeros_like(whole)
        for t in range(6):
            acc |= orc.coverage([12, 8, 5], P1[t:t + 1], P2[t:t + 1], crit)["bits"]
        assert np.array_equal(whole, acc)


def test_coverage_hand_built_cases(orc):
    # one layer of 3 then 2 neurons; pair 1: only neuron 1 of layer 1 flips,
    # and neuron 0 of layer 2 flips -> SS pair (1, 0); layer-2 neuron 1 has
    # ratio 4 -> SV pair (1, 1)
    a = np.array([5, -3, 7, 10, 2], np.int64)
    b = np.array([6, 3, 7, -10, 8], np.int64)
    ss = orc.coverage([3, 2], a[None], b[None], "SS")
    assert ss["covered_pairs"] == 1 and bit(ss["bits"], 1 * 2 + 0)
    sv = orc.coverage([3, 2], a[None], b[None], "SV")
    assert sv["covered_pairs"] == 1 and bit(sv["bits"], 1 * 2 + 1)
    # two flips in layer 1 -> no SS / SV at all
    b2 = np.array([-6, 3, 7, -10, 8], np.int64)
    assert orc.coverage([3, 2], a[None], b2[None], "SS")["covered_pairs"] == 0
    # no flip in layer 1, distance 1 >= 1 -> DS with layer-2 flips, all rows
    c = np.array([5, -3, 8, -10, 2], np.int64)
    ds = orc.coverage([3, 2], a[None], c[None], "DS", dist_sq_min=1)
    assert ds["covered_pairs"] == 3 and all(bit(ds["bits"], i * 2 + 0) for i in range(3))
    assert orc.coverage([3, 2], a[None], c[None], "DS", dist_sq_min=2)["covered_pairs"] == 0
    # zero potentials: sign(0) = 1, so 0 -> -1 flips and 0 -> 0 does not;
    # 0 vs 0 is no value change, 0 vs 5 is one
    z1 = np.array([0, 0, 1, 0, 0], np.int64)
    z2 = np.array([0, -1, 1, 0, 5], np.int64)
    r = orc.coverage([3, 2], z1[None], z2[None], "SV")
    assert r["covered_pairs"] == 1 and bit(r["bits"], 1 * 2 + 1)
