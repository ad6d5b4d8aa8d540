"""GPU parity of the integer lane-per-point enumeration (small networks) in
both domains against the oracle: the delta set (records identical to the
oracle's and to the matrix-core kernel's) and the L2 ball of Sec. III-C,
Eq. (9) (points per level, counterexamples, exact ties and every record
identical to the oracle's), including radii from the paper's Table III."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def same_as_oracle(s, cex, r):
    assert s["clean_label"] == r["clean_label"]
    assert list(s["points"]) == [int(v) for v in r["points"]]
    assert list(s["cex"]) == [int(v) for v in r["cex"]]
    assert list(s["ties"]) == [int(v) for v in r["ties"]]
    assert np.array_equal(cex["k"], r["cex_k"]) and np.array_equal(cex["rank"], r["cex_rank"])
    assert np.array_equal(cex["new_label"], r["cex_label"])


SHAPES = [
    (1, [35, 16, 5], 7),        # the C1 shape: 16-unit instance, one hidden layer
    (2, [20, 32, 10], 6),
    (3, [12, 64, 16], 6),       # 64 units, 16 classes
    (4, [35, 16, 8, 5], [6, 4]),
    (5, [30, 40, 30, 6], [6, 5]),
    (6, [64, 64, 64, 10], 5),
]


@pytest.mark.parametrize("seed,dims,shift", SHAPES)
def test_lane_kernel_delta_domain(ctx, orc, seed, dims, shift):
    """The default kernel for the shape (the lane kernel for one hidden
    layer of at most 16 units, else the matrix cores) and the lane kernel
    forced both return the oracle's records."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(700 + seed)
    net = I.random_qnet(g, dims, shift=shift, wmax=40, bmax=300)
    m = ibmc.Mlp(ctx, net)
    D = np.array([-90, -30, -5, 5, 30, 90], np.int16)
    x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    x[:3] = [0, 255, 128]
    r = orc.q8_check(net, x, D, 0, 2, cap=1 << 22)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 0, 2, cex_capacity=1 << 22)
    same_as_oracle(s, cex, r)
    ibmc.ibmc_set_variant(ctx, m, "lane")
    s2, cex2, _ = ibmc.ibmc_check_property(ctx, m, x, D, 0, 2, cex_capacity=1 << 22)
    same_as_oracle(s2, cex2, r)
    ibmc.ibmc_set_variant(ctx, m, None)


def test_some_delta_case_is_unsafe(orc):
    """The shapes above include counterexamples (so record emission is covered)."""
    hits = 0
    for seed, dims, shift in SHAPES:
        g = I.rng(700 + seed)
        net = I.random_qnet(g, dims, shift=shift, wmax=40, bmax=300)
        x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
        x[:3] = [0, 255, 128]
        hits += orc.q8_check(net, x, np.array([-90, -30, -5, 5, 30, 90], np.int16), 1, 2)["cex_total"] > 0
    assert hits >= 3


BALL_CASES = [
    (3, [35, 16, 5], 3, 400, 2),
    (1, [20, 32, 10], 5, 2000, 2),
    (6, [12, 64, 16], 3, 90, 3),
    (2, [35, 16, 8, 5], [3, 3], 1500, 2),
    (7, [30, 40, 30, 6], [5, 4], 50, 3),
    (2, [64, 64, 64, 10], [3, 3], 300, 2),
    (3, [35, 16, 5], 4, 5852, 2),    # the paper's smallest proximity, gamma = 0.3 (Table III): (0.3 * 255)^2
    (1, [10, 16, 4], 3, 70000, 2),   # radius above 255: offsets limited by the pixel range
]


def ball_case(seed, dims, shift):
    g = I.rng(800 + seed)
    net = I.random_qnet(g, dims, shift=shift, wmax=40, bmax=300)
    x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    x[:4] = [0, 255, 1, 254]
    return net, x


@pytest.mark.parametrize("seed,dims,shift,r2,kmax", BALL_CASES)
def test_ball_matches_oracle(ctx, orc, seed, dims, shift, r2, kmax):
    from paper_1907_12933_amd import ibmc
    net, x = ball_case(seed, dims, shift)
    m = ibmc.Mlp(ctx, net)
    print(f"ball {dims} r2={r2} k<={kmax}", flush=True)
    r = orc.q8_ball_check(net, x, r2, 0, kmax, cap=1 << 23)
    s, cex = ibmc.ibmc_check_ball(ctx, m, x, r2, 0, kmax, cex_capacity=1 << 23)
    same_as_oracle(s, cex, r)
    assert ibmc.ibmc_ball_digits(r2) * 2 == r["m"]


def test_ball_cases_are_unsafe(orc):
    """Every ball case above holds counterexamples, at the last level at least."""
    for seed, dims, shift, r2, kmax in BALL_CASES:
        net, x = ball_case(seed, dims, shift)
        r = orc.q8_ball_check(net, x, r2, 1, kmax)
        assert r["cex"][-1] > 0, dims


def test_ball_records_decode_into_the_ball(ctx):
    """Every record decodes (n_deltas = 2 rd) into an image inside [0, 255]^n
    within the radius, with exactly k changed pixels, whose label is the
    recorded one (replayed with the plain forward)."""
    from paper_1907_12933_amd import ibmc
    net, x = ball_case(3, [35, 16, 5], 4)
    m = ibmc.Mlp(ctx, net)
    r2 = 3000
    s, cex = ibmc.ibmc_check_ball(ctx, m, x, r2, 1, 2)
    assert len(cex) > 0
    Dv = ibmc.ball_deltas(r2)
    imgs = []
    for k, rank in zip(cex["k"], cex["rank"]):
        pix, dig = ibmc.ibmc_decode_point(35, len(Dv), int(k), int(rank))
        xp = x.astype(np.int64).copy()
        for p, d in zip(pix, dig):
            xp[p] += int(Dv[d])
        assert xp.min() >= 0 and xp.max() <= 255
        assert int(((xp - x) ** 2).sum()) <= r2 and int((xp != x).sum()) == k
        imgs.append(xp.astype(np.uint8))
    labels = ibmc.ibmc_forward(ctx, m, np.stack(imgs), want_potentials=False)
    assert np.array_equal(labels, cex["new_label"])


def test_ball_edges(ctx, orc):
    from paper_1907_12933_amd import ibmc
    net, x = ball_case(1, [20, 32, 10], 5)
    m = ibmc.Mlp(ctx, net)
    # radius 0: only the clean image
    s, cex = ibmc.ibmc_check_ball(ctx, m, x, 0, 0, 2)
    assert list(s["points"]) == [1, 0, 0] and s["cex_total"] == 0
    # an all-black image: negative offsets leave [0, 255]
    z = np.zeros(20, np.uint8)
    s, cex = ibmc.ibmc_check_ball(ctx, m, z, 200, 1, 2)
    r = orc.q8_ball_check(net, z, 200, 1, 2)
    same_as_oracle(s, cex, r)
    assert s["points"][0] == 20 * 14          # offsets 1..14 only
    # stop at the first unsafe level
    s, cex = ibmc.ibmc_check_ball(ctx, m, x, 2000, 1, 3, stop_at_first=True)
    r = orc.q8_ball_check(net, x, 2000, 1, 3, stop_at_first=True)
    same_as_oracle(s, cex, r)


def test_ball_batch_two_networks(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(903)
    n1 = I.random_qnet(g, [35, 16, 5], shift=3, wmax=40, bmax=300)
    n2 = I.random_qnet(g, [30, 40, 30, 6], shift=[5, 4], wmax=40, bmax=300)
    m1, m2 = ibmc.Mlp(ctx, n1), ibmc.Mlp(ctx, n2)
    xs = [g.integers(0, 255, size=35, endpoint=True).astype(np.uint8) for _ in range(3)]
    ys = [g.integers(0, 255, size=30, endpoint=True).astype(np.uint8) for _ in range(2)]
    props = [(m1, xs[0], 400, 1, 2), (m2, ys[0], 60, 0, 3), (m1, xs[1], 900, 1, 2), (m2, ys[1], 20, 1, 2),
             (m1, xs[2], 0, 1, 1)]
    refs = [(n1, xs[0], 400, 1, 2), (n2, ys[0], 60, 0, 3), (n1, xs[1], 900, 1, 2), (n2, ys[1], 20, 1, 2),
            (n1, xs[2], 0, 1, 1)]
    sums, cex = ibmc.ibmc_check_ball_batch(ctx, props, cex_capacity=1 << 22)
    for i, (net, x, r2, k0, k1) in enumerate(refs):
        r = orc.q8_ball_check(net, x, r2, k0, k1)
        same_as_oracle(sums[i], cex[cex["prop"] == i], r)


def test_ball_refusals(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(904)
    wide = ibmc.Mlp(ctx, I.random_qnet(g, [20, 128, 10], shift=6))
    x = g.integers(0, 255, size=20, endpoint=True).astype(np.uint8)
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_check_ball(ctx, wide, x, 100, 1, 2)
    assert e.value.code == ibmc.IBMC_E_UNIMPL
    fm = ibmc.Mlp(ctx, I.fnet_from_qnet(I.random_qnet(g, [20, 16, 5], shift=6)))
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_check_ball(ctx, fm, x, 100, 1, 2)
    assert e.value.code == ibmc.IBMC_E_UNIMPL
    small = ibmc.Mlp(ctx, I.random_qnet(g, [20, 16, 5], shift=6))
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_check_ball(ctx, small, x, -1, 1, 2)
    assert e.value.code == ibmc.IBMC_E_INVALID
