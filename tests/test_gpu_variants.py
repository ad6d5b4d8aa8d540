"""Every compiled instance of the integer enumeration kernel for the wide
shapes, forced in turn and compared with the oracle's exhaustive check of the
bounded domain (Sec. II-B: every image that differs from the clean one in k
pixels, k = 1..2, each shifted by a delta of the set), records bit-exact.

The shapes span hidden layers of 64 to 1024 units. That covers weights staged
in LDS and weights read through L2 (layers too large for LDS), one to four
16-point N-tiles per chunk, the fast and the general hidden requantiser, and
one and two hidden layers. The image of each network is the one of eight
seeded random images with the smallest clean margin, so that the domain
holds counterexamples."""
import json

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu

# (dims, shifts): shift[1] in {7, 8} takes the fast hidden requantiser,
# other values the general one
SHAPES = [
    ([64, 256, 256, 10], [7, 7]),
    ([64, 256, 256, 10], [7, 6]),
    ([64, 512, 256, 10], [7, 7]),
    ([64, 256, 512, 10], [7, 7]),
    ([64, 512, 512, 10], [7, 7]),
    ([64, 512, 512, 10], [7, 6]),
    ([64, 64, 512, 10], [7, 7]),
    ([64, 128, 512, 10], [7, 7]),
    ([64, 512, 64, 10], [7, 7]),
    ([64, 512, 128, 10], [7, 7]),
    ([64, 512, 10], [7]),
    ([64, 1024, 10], [7]),
]
DELTAS = np.array([-128, -64, 64, 128], np.int16)


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def narrow_image(net, g):
    """Of eight seeded images, the one whose two largest logits are closest."""
    from oracle import dense
    X = g.integers(0, 255, size=(8, net.dims[0]), endpoint=True).astype(np.uint8)
    z = np.sort(dense.q8_potentials(net, X)[:, -net.dims[-1]:], axis=1)
    return X[int(np.argmin(z[:, -1] - z[:, -2]))]


@pytest.mark.parametrize("dims,shift", SHAPES, ids=["-".join(map(str, d)) + f"_s{s[-1]}" for d, s in SHAPES])
def test_every_instance_matches_oracle(ctx, orc, dims, shift):
    from paper_1907_12933_amd import ibmc
    g = I.rng(sum(dims) + 31 * shift[-1])
    net = I.random_qnet(g, dims, shift=shift, wmax=16, bmax=2000)
    x = narrow_image(net, g)
    m = ibmc.Mlp(ctx, net)
    rep = json.loads(ibmc.ibmc_autotune(ctx, m, k=1, n_deltas=2))
    names = [v["name"] for v in rep["variants"]]
    ref = orc.q8_check(net, x, DELTAS, 1, 2)
    print(f"{dims} shift {shift}: {ref['cex_total']} counterexamples of {int(ref['points'].sum())} points; "
          f"instances {names}", flush=True)
    assert names
    try:
        for name in names:
            ibmc.ibmc_set_variant(ctx, m, name)
            assert ibmc.ibmc_chosen_variant(ctx, m) == name
            s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, DELTAS, 1, 2)
            assert s["cex_total"] == ref["cex_total"], name
            assert np.array_equal(cex["k"], ref["cex_k"]), name
            assert np.array_equal(cex["rank"], ref["cex_rank"]), name
            assert np.array_equal(cex["new_label"], ref["cex_label"]), name
    finally:
        ibmc.ibmc_set_variant(ctx, m, None)


# integer lane-per-point kernel: (first hidden, second hidden or 0, classes),
# padding to each of its instances (16|32|64, 0|16|32|64), some ragged
LANE_SHAPES = [(16, 0, 5), (30, 0, 10), (64, 0, 16), (16, 16, 5), (12, 30, 8), (16, 64, 10),
               (32, 16, 6), (32, 32, 10), (26, 48, 16), (64, 16, 7), (40, 32, 10), (64, 64, 16)]


@pytest.mark.parametrize("h1,h2,nc", LANE_SHAPES, ids=[f"lane-{a}-{b}-{c}" for a, b, c in LANE_SHAPES])
def test_every_lane_instance_matches_oracle(ctx, orc, h1, h2, nc):
    """The lane kernel forced on each of its instances: the label property
    and the threshold literal (V halfway between the two largest clean
    logits), records equal to the oracle's."""
    from paper_1907_12933_amd import ibmc
    dims = [30, h1] + ([h2] if h2 else []) + [nc]
    g = I.rng(500 + 7 * h1 + 3 * h2 + nc)
    net = I.random_qnet(g, dims, shift=[5] * (len(dims) - 2), wmax=40, bmax=300)
    x = narrow_image(net, g)
    D = np.array([-90, -40, 40, 90], np.int16)
    m = ibmc.Mlp(ctx, net)
    try:
        ibmc.ibmc_set_variant(ctx, m, "lane")
        assert ibmc.ibmc_chosen_variant(ctx, m) == "lane"
        s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
        ref = orc.q8_check(net, x, D, 1, 2)
        pot, _ = orc.q8_forward(net, x)
        z = np.sort(pot[-nc:])
        V = int(z[-2] + (z[-1] - z[-2]) // 2)
        sl, cexl, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2, literal_v=V)
        refl = orc.q8_check_literal(net, x, D, V, 1, 2)
    finally:
        ibmc.ibmc_set_variant(ctx, m, None)
    print(f"{dims}: {ref['cex_total']} counterexamples, {refl['cex_total']} literal violations", flush=True)
    assert ref["cex_total"] > 0
    for got, want in ((cex, ref), (cexl, refl)):
        assert np.array_equal(got["k"], want["cex_k"]) and np.array_equal(got["rank"], want["cex_rank"])
        assert np.array_equal(got["new_label"], want["cex_label"])
    assert list(s["ties"]) == [int(v) for v in ref["ties"]]
