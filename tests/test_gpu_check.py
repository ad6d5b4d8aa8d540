"""GPU parity of the exhaustive check against the CPU oracle, through the C ABI.

Integer work is compared bit for bit: clean label, per-level point /
counterexample / exact-tie counts, and the sorted (k, rank, new label)
records."""
import json

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu

D33 = np.arange(-16, 17, dtype=np.int16)


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def assert_same(s, cex, r):
    assert s["clean_label"] == r["clean_label"]
    assert list(s["levels"]) == list(r["levels"])
    assert list(s["points"]) == [int(v) for v in r["points"]]
    assert list(s["cex"]) == [int(v) for v in r["cex"]]
    assert list(s["ties"]) == [int(v) for v in r["ties"]]
    assert s["first_unsafe_k"] == r["first_unsafe_k"]
    n = min(len(cex), len(r["cex_rank"]))
    assert len(cex) == len(r["cex_rank"])
    assert np.array_equal(cex["k"][:n], r["cex_k"][:n])
    assert np.array_equal(cex["rank"][:n], r["cex_rank"][:n])
    assert np.array_equal(cex["new_label"][:n], r["cex_label"][:n])


def diff_net(w1=1, shift=0):
    return I.QNet([2, 2, 2], [np.array([[w1, 0], [0, w1]], np.int8), np.array([[1, -1], [-1, 1]], np.int8)],
                  [np.zeros(2, np.int32), np.zeros(2, np.int32)], [shift])


@pytest.mark.parametrize("x,w1,shift,deltas", [
    ((100, 90), 1, 0, D33), ((5, 10), 1, 0, D33), ((100, 90), 64, 7, D33), ((250, 240), 1, 0, D33),
    ((100, 90), 1, 0, np.array([-32, -16, -8, 8, 16, 32], np.int16))])
def test_closed_form_nets(ctx, orc, x, w1, shift, deltas):
    from paper_1907_12933_amd import ibmc
    net = diff_net(w1, shift)
    m = ibmc.Mlp(ctx, net)
    x = np.array(x, np.uint8)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, deltas, 0, 2)
    assert_same(s, cex, orc.q8_check(net, x, deltas, 0, 2))


@pytest.mark.parametrize("seed,dims,shift,wmax,k_max,deltas", [
    (1, [20, 12, 6], 3, 10, 3, [-60, -20, 20, 60]),
    (2, [24, 64, 16, 5], 4, 12, 2, [-48, -16, 16, 48]),
    (3, [30, 100, 70, 7], 5, 20, 2, [-40, -9, 0, 7, 33]),
    (4, [70, 64, 64, 10], 5, 16, 2, [-64, -32, 32, 64]),
    (5, [17, 130, 40, 3], 4, 10, 3, [-80, 80]),
    (6, [40, 200, 10], 4, 10, 2, [-50, -25, 25, 50]),
    # three layers with layer-2 shift 7 / 8 (the fast hidden requantiser); the
    # last two make every image a near tie (see below) for dense counterexamples
    (7, [40, 128, 64, 6], 7, 60, 2, [-60, -30, 30, 60]),
    (8, [48, 64, 192, 10], [7, 8], 64, 2, [-120, -60, 60, 120]),
    (9, [33, 256, 256, 10], [6, 7], 50, 2, [-100, -50, 50, 100]),
    # more than 16 classes: the output layer spans several M-tiles
    (10, [30, 64, 20], 4, 12, 2, [-60, -20, 20, 60]),
    (11, [24, 128, 64, 40], [5, 7], 20, 2, [-50, 50]),
    (12, [26, 64, 64, 17], 5, 16, 2, [-64, -32, 32, 64]),
])
def test_random_nets_full_lists(ctx, orc, seed, dims, shift, wmax, k_max, deltas):
    """Nets with dense counterexamples, several tiles and ragged tails: every
    record must match the oracle's."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(100 + seed)
    dense = seed in (7, 8, 9)
    net = I.random_qnet(g, dims, shift=shift, wmax=wmax, bmax=3000 if dense else 200)
    m = ibmc.Mlp(ctx, net)
    D = np.array(deltas, np.int16)
    for t in range(3):
        x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
        if seed in (8, 9):
            # move the runner-up logit to one below the top: many nearby points flip
            pot, lab = orc.q8_forward(net, x)
            z = pot[-dims[-1]:]
            j = int(np.argsort(z)[-2]) if int(np.argsort(z)[-1]) == lab else int(np.argsort(z)[-1])
            net.b[-1] = net.b[-1].copy()
            net.b[-1][j] += np.int32(z[lab] - z[j] - 1 - (1 if j < lab else 0))
            m = ibmc.Mlp(ctx, net)
        print(f"[check] seed={seed} dims={dims} image={t}", flush=True)
        s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 0, k_max)
        r = orc.q8_check(net, x, D, 0, k_max)
        assert_same(s, cex, r)


def test_glyph35_workload(ctx, orc):
    """35-16-5 net, ten 7x5 glyphs, deltas -16..16, k <= 2 (649,110 points per image)."""
    from paper_1907_12933_amd import ibmc
    w = I.workload_glyph35()
    m = ibmc.Mlp(ctx, w.net)
    props = [(m, w.images[i], w.deltas, 1, 2) for i in range(10)]
    sums, cex, _, rc = ibmc.ibmc_check_batch(ctx, props)
    for i in range(10):
        r = orc.q8_check(w.net, w.images[i], w.deltas, 1, 2)
        assert sums[i]["points_total"] == 649110
        assert sums[i]["clean_label"] == r["clean_label"]
        assert list(sums[i]["cex"]) == [int(v) for v in r["cex"]]
        sel = cex[cex["prop"] == i]
        assert np.array_equal(sel["rank"], r["cex_rank"]) and np.array_equal(sel["k"], r["cex_k"])


def test_batch_equals_single_calls(ctx, orc):
    """A batch over several nets and delta sets equals the per-property calls."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(77)
    nets = [I.random_qnet(g, [20, 12, 6], shift=3, wmax=10, bmax=200),
            I.random_qnet(g, [24, 64, 16, 5], shift=4, wmax=12, bmax=200)]
    ms = [ibmc.Mlp(ctx, n) for n in nets]
    props = []
    for t in range(6):
        ni = t % 2
        x = g.integers(0, 255, size=nets[ni].dims[0], endpoint=True).astype(np.uint8)
        D = np.array([[-60, -20, 20, 60], [-48, 48]][t % 2], np.int16)
        props.append((ms[ni], x, D, 1, 2 + (t % 2)))
    sums, cex, _, rc = ibmc.ibmc_check_batch(ctx, props)
    for i, (mm, x, D, k0, k1) in enumerate(props):
        r = orc.q8_check(nets[i % 2], x, D, k0, k1)
        sel = cex[cex["prop"] == i]
        assert list(sums[i]["cex"]) == [int(v) for v in r["cex"]]
        assert np.array_equal(sel["rank"], r["cex_rank"]) and np.array_equal(sel["new_label"], r["cex_label"])


def test_capacity_truncation_and_stop(ctx, orc):
    from paper_1907_12933_amd import ibmc
    net = diff_net()
    m = ibmc.Mlp(ctx, net)
    x = np.array([100, 90], np.uint8)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D33, 1, 2, cex_capacity=7)
    assert s["status"] == ibmc.IBMC_W_TRUNCATED and s["cex_total"] == 265 and len(cex) == 7
    # records kept under truncation are a subset of the true ones
    full = orc.q8_check(net, x, D33, 1, 2)
    keys = set(zip(full["cex_k"].tolist(), full["cex_rank"].tolist()))
    assert all((int(a), int(b)) in keys for a, b in zip(cex["k"], cex["rank"]))
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D33, 1, 2, stop_at_first=True)
    assert s["first_unsafe_k"] == 1 and s["levels"] == [1] and s["cex_total"] == 12


def test_replay_and_forward(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(5)
    net = I.random_qnet(g, [30, 100, 70, 7], shift=5, wmax=20, bmax=200)
    m = ibmc.Mlp(ctx, net)
    x = g.integers(0, 255, size=30, endpoint=True).astype(np.uint8)
    D = np.array([-40, -9, 0, 7, 33], np.int16)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
    assert len(cex) > 0
    lab = ibmc.ibmc_replay(ctx, m, x, D, cex)
    assert np.array_equal(lab, cex["new_label"])
    assert np.array_equal(orc.q8_eval_points(net, x, D, cex["k"], cex["rank"]), cex["new_label"])
    imgs = g.integers(0, 255, size=(9, 30), endpoint=True).astype(np.uint8)
    pots, labels = ibmc.ibmc_forward(ctx, m, imgs)
    for i in range(9):
        p, l = orc.q8_forward(net, imgs[i])
        assert np.array_equal(pots[i].astype(np.int64), p) and labels[i] == l


def test_load_errors(ctx):
    from paper_1907_12933_amd import ibmc
    big = I.QNet([3000, 4, 2], [np.ones((4, 3000), np.int8), np.ones((2, 4), np.int8)],
                 [np.zeros(4, np.int32), np.zeros(2, np.int32)], [0])
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.Mlp(ctx, big)
    assert e.value.code == ibmc.IBMC_E_UNIMPL
    # 2^31 - 100 + 255 reaches 2^31: rejected before any kernel runs
    rng_net = I.QNet([1, 4, 2], [np.ones((4, 1), np.int8), np.ones((2, 4), np.int8)],
                     [np.full(4, 2**31 - 100, np.int32), np.zeros(2, np.int32)], [0])
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.Mlp(ctx, rng_net)
    assert e.value.code == ibmc.IBMC_E_RANGE
    # shifts above 24 are refused (the kernels hold u - 64 * 2^s in int32)
    g = I.rng(3)
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.Mlp(ctx, I.random_qnet(g, [8, 16, 4], shift=25, wmax=8, bmax=8))
    assert e.value.code == ibmc.IBMC_E_INVALID
    # shift 24 with a bias of 2^30: |b| + 64 * 2^24 reaches 2^31 although
    # |b| + 255 sum|w| alone does not
    off = I.QNet([2, 2, 2], [np.ones((2, 2), np.int8), np.ones((2, 2), np.int8)],
                 [np.array([2**30, 0], np.int32), np.zeros(2, np.int32)], [24])
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.Mlp(ctx, off)
    assert e.value.code == ibmc.IBMC_E_RANGE


@pytest.mark.parametrize("seed,dims,shifts,bmax", [
    (42, [48, 64, 32, 6], [11, 9], 1 << 16),
    (59, [48, 64, 32, 6], [11, 9], 1 << 16),
    (7, [16, 32, 5], [24], 1 << 29),
])
def test_natural_large_shift(ctx, orc, seed, dims, shifts, bmax):
    """Shifts above 8 take the int32 first-layer path and the general
    requantiser on their own (no forcing); up to the largest accepted shift
    the records equal the oracle's."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.random_qnet(g, dims, shift=12, wmax=127, bmax=bmax)
    net.shift = list(shifts)
    x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    D = np.array([-255, -128, 128, 255], np.int16)
    m = ibmc.Mlp(ctx, net)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 0, 2)
    r = orc.q8_check(net, x, D, 0, 2)
    assert_same(s, cex, r)
    if seed in (42, 59):
        assert r["cex_total"] > 0


def test_general_first_layer_path(orc, monkeypatch):
    """The int32 first-layer path (taken when the packed int16 bound fails)
    gives the same records: forced on the same inputs, and reached naturally
    with deltas whose update bound exceeds the packed range."""
    from paper_1907_12933_amd import ibmc
    monkeypatch.setenv("IBMC_FIRST_LAYER", "int32")
    ctx32 = ibmc.Context(0)
    monkeypatch.delenv("IBMC_FIRST_LAYER")
    g = I.rng(31)
    net = I.random_qnet(g, [24, 64, 16, 5], shift=4, wmax=12, bmax=200)
    m = ibmc.Mlp(ctx32, net)
    D = np.array([-48, -16, 16, 48], np.int16)
    x = g.integers(0, 255, size=24, endpoint=True).astype(np.uint8)
    s, cex, _ = ibmc.ibmc_check_property(ctx32, m, x, D, 1, 2)
    assert_same(s, cex, orc.q8_check(net, x, D, 1, 2))
    # natural: 8-bit shift scale 2^(8-7)=2, |d| up to 200, |w| up to 64 -> 25600 > 8191
    net2 = I.random_qnet(g, [40, 64, 64, 10], shift=7, wmax=64, bmax=500)
    ctx = ibmc.Context(0)
    m2 = ibmc.Mlp(ctx, net2)
    D2 = np.array([-200, -100, 100, 200], np.int16)
    for t in range(2):
        x2 = g.integers(0, 255, size=40, endpoint=True).astype(np.uint8)
        s, cex, _ = ibmc.ibmc_check_property(ctx, m2, x2, D2, 1, 2)
        assert_same(s, cex, orc.q8_check(net2, x2, D2, 1, 2))


def test_fast_epilogue_headroom_gate(ctx, orc):
    """Layer-2 shift 7 selects the fast hidden epilogue only while every
    partial sum of its offset accumulators fits int32: a net whose layer-2
    bias is too large for it takes the general epilogue, with the same
    records as the oracle."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(161)
    net = I.random_qnet(g, [40, 64, 64, 6], shift=7, wmax=40, bmax=300)
    fast = ibmc.Mlp(ctx, net)
    big = I.random_qnet(I.rng(161), [40, 64, 64, 6], shift=7, wmax=40, bmax=300)
    big.b[1] = big.b[1].copy()
    big.b[1][3] = np.int32(1_100_000_000)    # alpha * (b + 256 sum|W|) + 32768 >= 2^31
    big.b[1][5] = np.int32(-1_100_000_000)
    slow = ibmc.Mlp(ctx, big)
    shape_fast = json.loads(ibmc.ibmc_autotune(ctx, fast, k=1, n_deltas=2))["shape"]
    shape_slow = json.loads(ibmc.ibmc_autotune(ctx, slow, k=1, n_deltas=2))["shape"]
    assert shape_fast.endswith("_f") and not shape_slow.endswith("_f")
    D = np.array([-60, -30, 30, 60], np.int16)
    for t in range(2):
        x = g.integers(0, 255, size=40, endpoint=True).astype(np.uint8)
        for net_, m in ((net, fast), (big, slow)):
            s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 0, 2)
            assert_same(s, cex, orc.q8_check(net_, x, D, 0, 2))
