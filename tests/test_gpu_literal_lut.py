"""GPU parity of the paper's threshold literal (Sec. III-C: the desired
class's output below the reference value V while another class's rises
above it) and of the table sigmoid (the sigmoid from a table, as the paper's
CUDA code did, Sec. IV-D), on the lane-per-point kernels, against the
oracle; and the count of the table's false and missed counterexamples
against the exact FP64 check (the threat to validity the paper names)."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def keys(ks, rs):
    return set(zip((int(a) for a in ks), (int(b) for b in rs)))


@pytest.mark.parametrize("dims,shift,seed", [([35, 16, 5], 4, 904), ([30, 40, 30, 6], [5, 4], 901)])
def test_integer_literal_matches_oracle(ctx, orc, dims, shift, seed):
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.random_qnet(g, dims, shift=shift, wmax=40, bmax=300)
    x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    pot, _ = orc.q8_forward(net, x)
    z = np.sort(pot[-dims[-1]:])
    V = int(z[-2] + (z[-1] - z[-2]) // 2)
    D = np.array([-90, -40, -10, 10, 40, 90], np.int16)
    m = ibmc.Mlp(ctx, net)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2, literal_v=V)
    r = orc.q8_check_literal(net, x, D, V, 1, 2)
    assert r["cex_total"] > 0
    assert list(s["cex"]) == [int(v) for v in r["cex"]] and list(s["ties"]) == [int(v) for v in r["ties"]]
    assert np.array_equal(cex["k"], r["cex_k"]) and np.array_equal(cex["rank"], r["cex_rank"])
    assert np.array_equal(cex["new_label"], r["cex_label"])
    # the label property of the same net and image is a different point set
    s2, cex2, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
    assert keys(cex2["k"], cex2["rank"]) != keys(cex["k"], cex["rank"])


@pytest.mark.parametrize("dims,seed,table", [([35, 16, 5], 910, False), ([35, 16, 5], 910, True),
                                             ([49, 128, 64, 10], 904, True)])
def test_float_literal_matches_oracle(ctx, orc, dims, seed, table):
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.fnet_from_qnet(I.random_qnet(g, dims, shift=7))
    x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    pot, _, _ = orc.f64_forward(net, x)
    z = np.sort(pot[-dims[-1]:])
    V = float((z[-1] + z[-2]) / 2)
    D = np.array([-64, -16, 16, 64], np.int16)
    m = ibmc.Mlp(ctx, net)
    s, cex, ties = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2, literal_v=V, table_sigmoid=table,
                                            near_tie_capacity=1 << 20)
    r = orc.f64_check(net, x, D, 1, 2, tie_rel=0.0, lut=table, literal_v=V)
    assert r["cex_total"] > 0
    diff = keys(cex["k"], cex["rank"]) ^ keys(r["cex_k"], r["cex_rank"])
    assert diff <= keys(ties["k"], ties["rank"])
    assert len(ties) <= max(10, r["cex_total"] // 10)


@pytest.mark.parametrize("dims,seed,differs", [([35, 16, 5], 25, True), ([35, 32, 16, 5], 72, True),
                                               ([49, 128, 64, 10], 5, False)])
def test_table_sigmoid_matches_oracle_and_counts_its_errors(ctx, orc, dims, seed, differs):
    """The table-sigmoid check equals the oracle's table-sigmoid check up to
    flagged near ties; against the exact FP64 check it adds and misses a
    few counterexamples (counted, each within the table's error of a tie)."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.fnet_from_qnet(I.random_qnet(g, dims, shift=7))
    x = I.glyph_images(g, 1, 7, 5)[0] if dims[0] == 35 else g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    D = np.arange(-16, 17, dtype=np.int16) if dims[0] == 35 else np.array([-64, -32, 32, 64], np.int16)
    m = ibmc.Mlp(ctx, net)
    s, cex, ties = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2, table_sigmoid=True, near_tie_capacity=1 << 20)
    ref_tab = orc.f64_check(net, x, D, 1, 2, tie_rel=0.0, lut=True)
    gpu = keys(cex["k"], cex["rank"])
    assert (gpu ^ keys(ref_tab["cex_k"], ref_tab["cex_rank"])) <= keys(ties["k"], ties["rank"])
    exact = orc.f64_check(net, x, D, 1, 2, tie_rel=0.0)
    ex = keys(exact["cex_k"], exact["cex_rank"])
    false_cex, missed = gpu - ex, ex - gpu
    print(f"table sigmoid {dims}: {len(gpu)} records, {len(false_cex)} false, {len(missed)} missed "
          f"against the exact check's {len(ex)}")
    assert (len(false_cex) + len(missed) > 0) == differs
    # every disagreement sits where the exact FP64 margin is below the
    # table's worst-case effect on the logits
    worst = 5e-5 * sum(float(np.abs(w).sum(axis=1).max()) for w in net.W[1:])
    pts = sorted(false_cex | missed)
    if pts:
        ks = np.array([k for k, _ in pts], np.int32)
        rs = np.array([r for _, r in pts], np.int64)
        _, _, mg = orc.f64_eval_points(net, x, D, ks, rs)
        assert np.all(mg <= 2 * worst + 1e-9)


def test_literal_and_table_refusals(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(77)
    wide = ibmc.Mlp(ctx, I.random_qnet(g, [20, 128, 10], shift=6))
    small = ibmc.Mlp(ctx, I.random_qnet(g, [20, 16, 5], shift=6))
    fwide = ibmc.Mlp(ctx, I.fnet_from_qnet(I.random_qnet(g, [20, 256, 10], shift=6)))
    x = g.integers(0, 255, size=20, endpoint=True).astype(np.uint8)
    D = np.array([-40, 40], np.int16)
    cases = [(wide, dict(literal_v=10), ibmc.IBMC_E_UNIMPL),
             (small, dict(table_sigmoid=True), ibmc.IBMC_E_INVALID),
             (small, dict(literal_v=1.5), ibmc.IBMC_E_INVALID),
             (small, dict(literal_v=10, chunk_budget=5), ibmc.IBMC_E_UNIMPL),
             (fwide, dict(table_sigmoid=True), ibmc.IBMC_E_UNIMPL)]
    for m, kw, code in cases:
        with pytest.raises(ibmc.IbmcError) as e:
            ibmc.ibmc_check_property(ctx, m, x, D, 1, 2, **kw)
        assert e.value.code == code, kw
