"""GPU parity of the FP32 sigmoid variant against the FP64 oracle.

The bar (float variant, Sec. II-A Eqs. (1)-(2)):
  - the enumeration's own logits (read back for listed points through
    ibmc_eval_points_f32, which repeats the enumeration kernels' arithmetic)
    stay within 1e-5 * max(1, |z64|) of the FP64 oracle on every
    counterexample, every flagged point and at least 10^5 seeded points per
    property, up to 784-512-512-10;
  - the eval arithmetic is the enumeration's: a listed point is a record iff
    its eval label differs from the clean label, with the same label;
  - every point whose FP32 decision differs from the FP64 decision is in the
    near-tie list, and a flagged point's FP64 margin is small (the flags are
    not spurious);
  - logits of the plain FP32 forward stay within the same tolerance."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu

D33 = np.arange(-16, 17, dtype=np.int16)
EPS = 1e-5          # per-logit tolerance relative to max(1, |z64|)
TAU = 4e-5          # the library's default near-tie threshold


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def keyset(ks, rs):
    return set(zip((int(a) for a in ks), (int(b) for b in rs)))


def check_against_fp64(ibmc, ctx, orc, net, x, D, k_max):
    m = ibmc.Mlp(ctx, net)
    s, cex, ties = ibmc.ibmc_check_property(ctx, m, x, D, 1, k_max, near_tie_capacity=1 << 20)
    r = orc.f64_check(net, x, D, 1, k_max, tie_rel=0.0)
    assert s["clean_label"] == r["clean_label"]
    gpu = keyset(cex["k"], cex["rank"])
    ref = keyset(r["cex_k"], r["cex_rank"])
    flagged = keyset(ties["k"], ties["rank"])
    assert len(ties) == s["near_ties_total"]
    diff = gpu ^ ref
    assert diff <= flagged, f"{len(diff - flagged)} decisions differ without a near-tie flag"
    return s, gpu, ref, flagged


def test_closed_form_float(ctx, orc):
    from paper_1907_12933_amd import ibmc
    net = I.FNet([2, 2, 2], [np.eye(2, dtype=np.float32), np.array([[1, -1], [-1, 1]], np.float32)],
                 [np.zeros(2, np.float32), np.zeros(2, np.float32)])
    x = np.array([100, 90], np.uint8)
    s, gpu, ref, flagged = check_against_fp64(ibmc, ctx, orc, net, x, D33, 2)
    # margin-zero points (x0' == x1') are ties: 2 at k=1, 23 at k=2, all flagged
    assert s["ties"] == [2, 23]
    assert len(ref) == 12 + 253 and gpu == ref


@pytest.mark.parametrize("seed,dims,k_max,deltas", [
    (1, [35, 16, 5], 2, D33),
    (2, [64, 32, 10], 2, np.array([-32, -16, 16, 32], np.int16)),
    (3, [100, 64, 10], 2, np.array([-64, 64], np.int16)),
    (4, [35, 32, 16, 5], 3, np.array([-100, 100], np.int16)),
    (5, [49, 128, 64, 10], 2, np.array([-64, 64], np.int16)),     # widest one-point-per-lane shape
    (6, [40, 200, 10], 2, np.array([-80, 80], np.int16)),         # sixteen points per wave
    (7, [30, 40, 30, 20, 5], 2, np.array([-90, 90], np.int16)),   # three hidden layers
])
def test_random_float_nets(ctx, orc, seed, dims, k_max, deltas):
    from paper_1907_12933_amd import ibmc
    g = I.rng(300 + seed)
    q = I.random_qnet(g, dims, shift=7)
    net = I.fnet_from_qnet(q)
    for t in range(2):
        x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
        _, lab, mg = orc.f64_forward(net, x)
        if mg < 1e-3:
            continue          # the clean decision itself is a near tie
        check_against_fp64(ibmc, ctx, orc, net, x, deltas, k_max)


@pytest.mark.parametrize("seed,dims,deltas", [
    (21, [35, 16, 5], D33),
    (22, [196, 128, 64, 10], np.array([-32, -16, 16, 32], np.int16)),
    (23, [784, 256, 256, 10], np.array([-32, 32], np.int16)),
    (24, [784, 512, 512, 10], np.array([-32, 32], np.int16)),
])
def test_enumeration_logits_within_tolerance(ctx, orc, seed, dims, deltas):
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.fnet_from_qnet(I.random_qnet(g, dims, shift=7))
    n = dims[0]
    x = I.glyph_images(g, 1, 7, 5)[0] if n == 35 else I.blob_images(g, 1, {196: 14, 784: 28}[n])[0]
    m = ibmc.Mlp(ctx, net)
    print(f"float tolerance: {dims} k=1..2", flush=True)
    s, cex, ties = ibmc.ibmc_check_property(ctx, m, x, deltas, 1, 2, cex_capacity=1 << 21,
                                            near_tie_capacity=1 << 20)
    assert s["cex_total"] <= (1 << 21) and s["near_ties_total"] <= (1 << 20)
    M = len(deltas)
    n1, n2 = orc.points(n, M, 1), orc.points(n, M, 2)
    samp = g.integers(0, n2, 100_000)
    ks = np.concatenate([np.ones(n1, np.int32), np.full(samp.size, 2, np.int32), cex["k"], ties["k"]])
    ranks = np.concatenate([np.arange(n1), samp, cex["rank"], ties["rank"]]).astype(np.int64)
    z32, lab32, mg32, clean32 = ibmc.ibmc_eval_points_f32(ctx, m, x, deltas, ks, ranks)
    lab64, z64, mg64 = orc.f64_eval_points(net, x, deltas, ks, ranks)
    rel = np.abs(z32.astype(np.float64) - z64) / np.maximum(1.0, np.abs(z64))
    assert rel.max() <= EPS, (dims, float(rel.max()))
    # the listed points are evaluated by the enumeration's arithmetic
    assert clean32 == s["clean_label"]
    recs = keyset(cex["k"], cex["rank"])
    flagged = keyset(ties["k"], ties["rank"])
    nl = n1 + samp.size
    for t in range(nl):
        assert ((lab32[t] != clean32) == ((int(ks[t]), int(ranks[t])) in recs)), t
    nc = len(cex)
    assert np.array_equal(lab32[nl:nl + nc], cex["new_label"])
    # decisions that differ from FP64 carry a near-tie flag
    _, clean64, _ = orc.f64_forward(net, x)
    assert clean64 == clean32
    for t in np.nonzero(lab32[:nl] != lab64[:nl])[0]:
        assert (int(ks[t]), int(ranks[t])) in flagged
    # flags are not spurious: a flagged point's FP64 margin is within the
    # threshold plus twice the logit tolerance
    ft = slice(nl + nc, None)
    top64 = np.max(z64[ft], axis=1) if len(ties) else np.zeros(0)
    assert np.all(mg64[ft] <= (TAU + 2 * EPS) * np.maximum(1.0, np.abs(top64)) * 1.01)


def test_eval_points_errors(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(77)
    qn = I.random_qnet(g, [35, 16, 5], shift=7)
    fm = ibmc.Mlp(ctx, I.fnet_from_qnet(qn))
    x = I.glyph_images(g, 1, 7, 5)[0]
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_eval_points_f32(ctx, fm, x, D33, [2], [595 * 33 * 33])
    assert e.value.code == ibmc.IBMC_E_INVALID
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_eval_points_f32(ctx, ibmc.Mlp(ctx, qn), x, D33, [1], [0])
    assert e.value.code == ibmc.IBMC_E_UNIMPL
    # k = 0 is the clean image itself
    z, lab, mg, clean = ibmc.ibmc_eval_points_f32(ctx, fm, x, D33, [0], [0])
    assert lab[0] == clean


def test_float_logits_tolerance(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(311)
    for dims in ([784, 256, 256, 10], [196, 128, 64, 10], [35, 16, 5]):
        net = I.fnet_from_qnet(I.random_qnet(g, dims, shift=7))
        m = ibmc.Mlp(ctx, net)
        imgs = g.integers(0, 255, size=(64, dims[0]), endpoint=True).astype(np.uint8)
        pots, labels = ibmc.ibmc_forward(ctx, m, imgs)
        worst = 0.0
        for i in range(64):
            p, lab, mg = orc.f64_forward(net, imgs[i])
            z32 = pots[i][-dims[-1]:].astype(np.float64)
            z64 = p[-dims[-1]:]
            worst = max(worst, float(np.max(np.abs(z32 - z64) / np.maximum(1.0, np.abs(z64)))))
            if mg > 1e-4:
                assert labels[i] == lab
        assert worst <= 1e-5, (dims, worst)
