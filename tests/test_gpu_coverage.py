"""GPU parity of the coverage criteria against the CPU oracle through the C
ABI: the paper's worked tables from potentials, and full networks from
images (potentials from the batched int8 MFMA forward)."""
import os

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CRITS = ["SS", "DS", "SV", "DV"]


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def same(gpu, ref):
    for key in ("covered_pairs", "total_pairs", "covered_neurons", "total_neurons", "literal"):
        assert gpu[key] == ref[key], (key, gpu[key], ref[key])
    assert abs(gpu["fraction"] - ref["fraction"]) < 1e-12
    assert np.array_equal(gpu["bits"], ref["bits"])


def test_table1_from_potentials(ctx, orc):
    from paper_1907_12933_amd import ibmc
    pots = {r[0]: np.array([int(v) for v in r[2:]], np.int64) for r in rows("table1_potentials.txt")}
    for crit, pair, npairs, nneur, _ in rows("table1_coverage.txt"):
        a, b = pair.split(",")
        g = ibmc.ibmc_coverage_from_potentials(ctx, [3, 2, 1], pots[a], pots[b], crit, dist_sq_min=10000)
        r = orc.coverage([3, 2, 1], pots[a][None], pots[b][None], crit, dist_sq_min=10000)
        same(g, r)
        assert g["covered_pairs"] == int(npairs) and g["covered_neurons"] == int(nneur)


def test_table2_from_potentials(ctx, orc):
    from paper_1907_12933_amd import ibmc
    rr = rows("table2_potentials.txt")
    u = np.array([int(r[1]) for r in rr], np.int64)
    v = np.array([int(r[2]) for r in rr], np.int64)
    g = ibmc.ibmc_coverage_from_potentials(ctx, [5, 4, 5], u, v, "SS", P=0.8)
    assert g["covered_pairs"] == 2 and g["covered_neurons"] == 3 and g["total_neurons"] == 14
    assert g["literal"] is False
    for crit in CRITS:
        same(ibmc.ibmc_coverage_from_potentials(ctx, [5, 4, 5], u, v, crit),
             orc.coverage([5, 4, 5], u[None], v[None], crit))


def test_forward_potentials_exact(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(8)
    for dims in ([35, 16, 5], [784, 256, 256, 10], [100, 1024, 64, 1000 // 100], [60, 130, 70, 40, 7]):
        net = I.random_qnet(g, dims, shift=7)
        m = ibmc.Mlp(ctx, net)
        imgs = g.integers(0, 255, size=(37, dims[0]), endpoint=True).astype(np.uint8)
        pots, labels = ibmc.ibmc_forward(ctx, m, imgs)
        for i in range(37):
            p, lab = orc.q8_forward(net, imgs[i])
            assert np.array_equal(pots[i].astype(np.int64), p), (dims, i)
            assert labels[i] == lab


@pytest.mark.parametrize("seed,dims,shift,pairs,maxpix,maxshift,dmin", [
    (1, [20, 12, 8, 5], 4, 40, 6, 40, 1),
    (2, [35, 16, 5], 7, 100, 8, 16, 1),
    (3, [64, 70, 33, 10], 5, 60, 8, 64, 50),
    (4, [30, 100, 90, 80, 6], 4, 30, 3, 90, 1),
    # widths whose 16-row tiles split evenly over the eight waves: one, two
    # and four tiles per wave (128, 256, 512 units)
    (5, [40, 128, 256, 10], 6, 24, 6, 64, 50),
    (6, [40, 512, 128, 10], 6, 24, 6, 64, 50),
])
def test_random_nets_all_criteria(ctx, orc, seed, dims, shift, pairs, maxpix, maxshift, dmin):
    from paper_1907_12933_amd import ibmc
    import torch
    g = I.rng(200 + seed)
    net = I.random_qnet(g, dims, shift=shift, wmax=20, bmax=300)
    x1 = g.integers(0, 255, size=(pairs, dims[0]), endpoint=True).astype(np.uint8)
    x2 = np.stack([I.perturbed_partner(g, x, maxpix, maxshift) for x in x1])
    m = ibmc.Mlp(ctx, net)
    P1 = np.stack([orc.q8_forward(net, x)[0] for x in x1])
    P2 = np.stack([orc.q8_forward(net, x)[0] for x in x2])
    widths = dims[1:]
    refs = [orc.coverage(widths, P1, P2, c, dist_sq_min=dmin) for c in CRITS]
    for c, ref in zip(CRITS, refs):
        same(ibmc.ibmc_coverage(ctx, m, x1, x2, c, dist_sq_min=dmin), ref)
    d1 = torch.from_numpy(x1).cuda(); d2 = torch.from_numpy(x2).cuda()
    for got, ref in zip(ibmc.ibmc_coverage_all_dev(ctx, m, d1, d2, dist_sq_min=dmin), refs):
        same(got, ref)


def test_glyph35_coverage_pairs(ctx, orc):
    """35-16-5 net, 100 seeded pairs (x2 = x1 with 1-8 pixels shifted)."""
    from paper_1907_12933_amd import ibmc
    net, x1, x2 = I.coverage_pairs_glyph35()
    m = ibmc.Mlp(ctx, net)
    P1 = np.stack([orc.q8_forward(net, x)[0] for x in x1])
    P2 = np.stack([orc.q8_forward(net, x)[0] for x in x2])
    for c in CRITS:
        same(ibmc.ibmc_coverage(ctx, m, x1, x2, c), orc.coverage([16, 5], P1, P2, c))


def test_wide_net_sampled_pairs(ctx, orc):
    """784-1024-1024-1024-10 net on a seeded subset of its pairs (the oracle
    evaluates every neuron pair literally)."""
    from paper_1907_12933_amd import ibmc
    net, x1, x2 = I.coverage_pairs_blob784(n_pairs=48)
    m = ibmc.Mlp(ctx, net)
    P1 = np.stack([orc.q8_forward(net, x)[0] for x in x1])
    P2 = np.stack([orc.q8_forward(net, x)[0] for x in x2])
    for c in CRITS:
        same(ibmc.ibmc_coverage(ctx, m, x1, x2, c), orc.coverage([1024, 1024, 1024, 10], P1, P2, c))


def test_coverage_invariants(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(9)
    net = I.random_qnet(g, [40, 64, 32, 8], shift=4, wmax=20, bmax=300)
    m = ibmc.Mlp(ctx, net)
    x1 = g.integers(0, 255, size=(30, 40), endpoint=True).astype(np.uint8)
    x2 = np.stack([I.perturbed_partner(g, x, 5, 60) for x in x1])
    for c in CRITS:
        a = ibmc.ibmc_coverage(ctx, m, x1, x2, c)
        b = ibmc.ibmc_coverage(ctx, m, x2, x1, c)
        assert np.array_equal(a["bits"], b["bits"])
        z = ibmc.ibmc_coverage(ctx, m, x1, x1, c)
        assert z["covered_pairs"] == 0 and z["covered_neurons"] == 0


@pytest.mark.parametrize("ndiff", [[16, 1, 3], [17, 2, 0], [40, 5, 16], [None]])
def test_pair_rank_update_and_dense_tiles(ctx, orc, ndiff):
    """x2's first layer is the rank-r update of x1's when every pair of a
    16-pair tile differs in at most 16 pixels, else the tile's x2 images run
    the full first layer: pairs differing in 0, 1, 16, 17, 40 or every
    pixel, mixed within tiles, against the oracle."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(300 + len(ndiff) + (ndiff[0] or 0))
    dims = [50, 70, 33, 9]
    net = I.random_qnet(g, dims, shift=5, wmax=20, bmax=300)
    m = ibmc.Mlp(ctx, net)
    n_pairs = 45
    x1 = g.integers(0, 255, size=(n_pairs, 50), endpoint=True).astype(np.uint8)
    x2 = x1.copy()
    for i in range(n_pairs):
        k = ndiff[i % len(ndiff)]
        if k is None:
            x2[i] = g.integers(0, 255, size=50, endpoint=True)
            continue
        pix = g.choice(50, size=k, replace=False)
        x2[i, pix] = (x1[i, pix].astype(np.int64) + g.integers(1, 255, size=k)) % 256
    P1 = np.stack([orc.q8_forward(net, x)[0] for x in x1])
    P2 = np.stack([orc.q8_forward(net, x)[0] for x in x2])
    for c in CRITS:
        same(ibmc.ibmc_coverage(ctx, m, x1, x2, c, dist_sq_min=100), orc.coverage(dims[1:], P1, P2, c, dist_sq_min=100))
