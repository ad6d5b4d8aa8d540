"""Batched uneven properties: eight networks 35-16-5 ... 784-512-512-10,
per-property k and delta sets, all in one captured graph of persistent
launches; compared property by property with the oracle, replayed several
times against the eager single-property results."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


@pytest.fixture(scope="module")
def small_batch():
    # same generator as the full 256-property workload, with an oracle budget
    # that keeps the CPU side to seconds
    return I.batch_workload(seed=3, per_net=2, mac_budget=3e9)


def test_batch_matches_oracle_and_replays(ctx, orc, small_batch):
    from paper_1907_12933_amd import ibmc
    nets, props = small_batch
    ms = [ibmc.Mlp(ctx, n) for n in nets]
    P = [(ms[p.net_index], p.image, p.deltas, 1, p.k) for p in props]
    first = None
    for rep in range(3):
        sums, cex, _, rc = ibmc.ibmc_check_batch(ctx, P)
        # eager work between graph replays
        s0, c0, _ = ibmc.ibmc_check_property(ctx, ms[props[0].net_index], props[0].image, props[0].deltas, 1,
                                             props[0].k)
        assert list(s0["cex"]) == list(sums[0]["cex"])
        if first is None:
            first = (sums, cex)
            for i, p in enumerate(props):
                r = orc.q8_check(nets[p.net_index], p.image, p.deltas, 1, p.k)
                assert sums[i]["clean_label"] == r["clean_label"], i
                assert list(sums[i]["points"]) == [int(v) for v in r["points"]], i
                assert list(sums[i]["cex"]) == [int(v) for v in r["cex"]], i
                sel = cex[cex["prop"] == i]
                assert np.array_equal(sel["rank"], r["cex_rank"]) and np.array_equal(sel["k"], r["cex_k"]), i
                assert np.array_equal(sel["new_label"], r["cex_label"]), i
        else:
            assert np.array_equal(cex, first[1])
            assert [s["cex"] for s in sums] == [s["cex"] for s in first[0]]


def test_mixed_integer_and_float_batch(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(55)
    q1 = I.random_qnet(g, [35, 16, 5], shift=4, wmax=20, bmax=200)
    q2 = I.random_qnet(g, [64, 32, 10], shift=7)
    f2 = I.fnet_from_qnet(q2)
    m1, m2 = ibmc.Mlp(ctx, q1), ibmc.Mlp(ctx, f2)
    x1 = I.glyph_images(g, 1, 7, 5)[0]
    x2 = g.integers(0, 255, size=64, endpoint=True).astype(np.uint8)
    D1 = np.array([-60, -20, 20, 60], np.int16)
    D2 = np.array([-48, -16, 16, 48], np.int16)
    sums, cex, ties, rc = ibmc.ibmc_check_batch(ctx, [(m1, x1, D1, 1, 2), (m2, x2, D2, 1, 2)],
                                                near_tie_capacity=1 << 16)
    r1 = orc.q8_check(q1, x1, D1, 1, 2)
    assert list(sums[0]["cex"]) == [int(v) for v in r1["cex"]]
    assert np.array_equal(cex[cex["prop"] == 0]["rank"], r1["cex_rank"])
    r2 = orc.f64_check(f2, x2, D2, 1, 2, tie_rel=0.0)
    gpu = set(zip(cex[cex["prop"] == 1]["k"].tolist(), cex[cex["prop"] == 1]["rank"].tolist()))
    ref = set(zip(r2["cex_k"].tolist(), r2["cex_rank"].tolist()))
    flagged = set(zip(ties["k"].tolist(), ties["rank"].tolist()))
    assert (gpu ^ ref) <= flagged


def test_autotune_picks_a_working_variant(ctx, orc):
    from paper_1907_12933_amd import ibmc
    import json
    g = I.rng(56)
    net = I.random_qnet(g, [64, 64, 64, 10], shift=5, wmax=16, bmax=200)
    m = ibmc.Mlp(ctx, net)
    rep = json.loads(ibmc.ibmc_autotune(ctx, m, k=2, n_deltas=4))
    assert rep["best"] in [v["name"] for v in rep["variants"]] and len(rep["variants"]) >= 2
    x = g.integers(0, 255, size=64, endpoint=True).astype(np.uint8)
    D = np.array([-64, -32, 32, 64], np.int16)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
    r = orc.q8_check(net, x, D, 1, 2)
    assert np.array_equal(cex["rank"], r["cex_rank"])
    for v in rep["variants"]:
        ibmc.ibmc_set_variant(ctx, m, v["name"])
        s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
        assert np.array_equal(cex["rank"], r["cex_rank"]) and np.array_equal(cex["new_label"], r["cex_label"]), v
    ibmc.ibmc_set_variant(ctx, m, None)


def test_records_on_device_match_host(ctx, small_batch):
    """Device-resident record output (images and records in HBM) hands out
    the same sorted records and totals as the host-buffer path, with and
    without truncation."""
    import torch
    from paper_1907_12933_amd import ibmc
    nets, props = small_batch
    ms = [ibmc.Mlp(ctx, n) for n in nets]
    imgs = [torch.from_numpy(np.ascontiguousarray(p.image)).cuda() for p in props]
    P = [(ms[p.net_index], imgs[i], p.deltas, 1, p.k) for i, p in enumerate(props)]
    for cap in (1 << 20, 5):
        s1, c1, _, rc1 = ibmc.ibmc_check_batch_dev(ctx, P, cex_capacity=cap)
        s2, c2, _, rc2 = ibmc.ibmc_check_batch_dev(ctx, P, cex_capacity=cap, records_on_device=True)
        assert rc1 == rc2 and [s["cex"] for s in s1] == [s["cex"] for s in s2]
        host = np.frombuffer(c2.cpu().numpy().tobytes(), dtype=ibmc.CEX_DTYPE)
        assert len(host) == len(c1) == min(cap, sum(s["cex_total"] for s in s1))
        if cap > 5:
            assert np.array_equal(host, c1)


def test_tuning_table_drives_the_batch_and_the_graph_replays(ctx, orc, tmp_path):
    """Tuned choices are saved, loaded into a fresh context and launched by
    the batched check (the chosen kernel is the table's, including a table
    that sends a two-layer network to the lane kernel); a repeated batch
    replays its instantiated graph; every call returns the oracle's records."""
    from paper_1907_12933_amd import ibmc
    import json
    g = I.rng(57)
    n1 = I.random_qnet(g, [35, 16, 5], shift=4, wmax=40, bmax=300)
    n2 = I.random_qnet(g, [30, 40, 30, 6], shift=[5, 4], wmax=40, bmax=300)
    c1 = ibmc.Context(0)
    m1, m2 = ibmc.Mlp(c1, n1), ibmc.Mlp(c1, n2)
    best = {}
    for m in (m1, m2):
        rep = json.loads(ibmc.ibmc_autotune(c1, m, k=2, n_deltas=6))
        best[rep["shape"]] = rep["best"]
        assert ibmc.ibmc_chosen_variant(c1, m) == rep["best"]
    path = tmp_path / "tune.json"
    ibmc.ibmc_tune_save(c1, path)
    del m1, m2
    c1.close()
    assert json.loads(path.read_text()) == best
    D = np.array([-90, -30, 30, 90], np.int16)
    xs = [g.integers(0, 255, size=35, endpoint=True).astype(np.uint8) for _ in range(2)]
    ys = [g.integers(0, 255, size=30, endpoint=True).astype(np.uint8) for _ in range(2)]
    refs = [orc.q8_check(n1, xs[0], D, 1, 2), orc.q8_check(n2, ys[0], D, 1, 2), orc.q8_check(n1, xs[1], D, 1, 2),
            orc.q8_check(n2, ys[1], D, 1, 2)]
    assert sum(r["cex_total"] > 0 for r in refs) >= 2
    for table in (best, {k: ("lane" if k.startswith("q8_30_") else v) for k, v in best.items()}):
        path.write_text(json.dumps(table))
        c2 = ibmc.Context(0)
        assert ibmc.ibmc_tune_load(c2, path) == 2
        a1, a2 = ibmc.Mlp(c2, n1), ibmc.Mlp(c2, n2)
        assert [ibmc.ibmc_chosen_variant(c2, a) for a in (a1, a2)] == list(table.values())
        props = [(a1, xs[0], D, 1, 2), (a2, ys[0], D, 1, 2), (a1, xs[1], D, 1, 2), (a2, ys[1], D, 1, 2)]
        l0, r0 = ibmc.ibmc_graph_stats(c2)
        outs = [ibmc.ibmc_check_batch(c2, props, cex_capacity=1 << 20) for _ in range(3)]
        l1, r1 = ibmc.ibmc_graph_stats(c2)
        assert l1 - l0 == 3 and r1 - r0 == 2
        for sums, cex, _, _ in outs:
            for i, r in enumerate(refs):
                c = cex[cex["prop"] == i]
                assert list(sums[i]["cex"]) == [int(v) for v in r["cex"]]
                assert np.array_equal(c["rank"], r["cex_rank"]) and np.array_equal(c["new_label"], r["cex_label"])
        c2.close()
