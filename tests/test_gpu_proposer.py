"""GPU parity of the learned proposal network: features against the oracle,
bf16 MFMA gradients against the FP64 oracle gradients, training, the
ordering by score, and the ordered search keeping the plain verdicts."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def bf16_round(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_features_match_oracle(ctx, orc):
    from paper_1907_12933_amd import ibmc
    w = I.workload_blob784(count=3)
    m = ibmc.Mlp(ctx, w.net)
    for i in range(3):
        g = ibmc.ibmc_proposer_features(ctx, m, w.images[i], 28, 28, w.deltas)
        r = orc.prop_features(w.net, w.images[i], 28, 28, w.deltas)
        np.testing.assert_allclose(g, r, rtol=2e-6, atol=1e-7)


def test_gradients_match_fp64(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(17)
    prop = ibmc.Proposer(ctx, seed=3)
    W1, b1, w2, c = prop.get()
    b1 = (g.normal(size=128) * 0.2).astype(np.float32)
    c = 0.1
    prop.set(W1, b1, w2, c)
    for B in (64, 1000, 4096):
        f = g.random((B, 32)).astype(np.float32)
        f[:, 9:] = 0.0
        y = (g.random(B) < 0.2).astype(np.float32)
        pw = 3.0
        got = ibmc.ibmc_proposer_grad(ctx, prop, f, y, pw)
        ref = orc.prop_loss_grad(bf16_round(f), y.astype(np.float64), pw, bf16_round(W1), b1.astype(np.float64),
                                 w2.astype(np.float64), float(c))
        assert abs(got["loss"] - ref["loss"]) <= 2e-3 * abs(ref["loss"])
        for k in ("W1", "b1", "w2"):
            a, b = got[k].astype(np.float64).ravel(), ref[k].ravel()
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            assert rel <= 2e-2 and cos >= 0.999, (B, k, rel, cos)
        assert abs(got["c"] - ref["c"]) <= 2e-3 * max(abs(ref["c"]), 1e-3)


def test_training_learns_separable_labels(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(21)
    N = 20000
    f = g.random((N, 32)).astype(np.float32)
    f[:, 9:] = 0.0
    f[:, 8] = 1.0
    y = ((f[:, 0] + 0.5 * f[:, 4] - 0.3 * f[:, 2]) > 0.9).astype(np.float32)
    prop = ibmc.Proposer(ctx, seed=5)
    losses = ibmc.ibmc_proposer_train(ctx, prop, f, y, epochs=15, batch=1024, lr=3e-3, seed=9)
    assert losses[-1] < 0.5 * losses[0]
    # the learned scores rank positives first (AUC)
    from paper_1907_12933_amd.ibmc import PROP_FEATURES  # noqa: F401
    W1, b1, w2, c = prop.get()
    h = np.maximum(f.astype(np.float64) @ W1.T.astype(np.float64) + b1, 0)
    s = h @ w2 + c
    pos, neg = s[y > 0.5], s[y < 0.5]
    auc = (np.searchsorted(np.sort(neg), pos).sum()) / (len(pos) * len(neg))
    assert auc > 0.95


def test_ranked_search_keeps_the_plain_verdicts(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(41)
    net = I.random_qnet(g, [64, 64, 64, 10], shift=5, wmax=16, bmax=200)
    m = ibmc.Mlp(ctx, net)
    D = np.array([-64, -32, 32, 64], np.int16)
    prop = ibmc.Proposer(ctx, seed=1)
    for t in range(3):
        x = g.integers(0, 255, size=64, endpoint=True).astype(np.uint8)
        plain, pc = ibmc.ibmc_check_property_ranked(ctx, m, None, x, 8, 8, D, 1, 2)
        ranked, rc = ibmc.ibmc_check_property_ranked(ctx, m, prop, x, 8, 8, D, 1, 2)
        ref = orc.q8_check(net, x, D, 1, 2)
        for s, cx in ((plain, pc), (ranked, rc)):
            assert list(s["cex"]) == [int(v) for v in ref["cex"]]
            assert np.array_equal(cx["rank"], ref["cex_rank"]) and np.array_equal(cx["k"], ref["cex_k"])
            assert np.array_equal(cx["new_label"], ref["cex_label"])
            if ref["cex_total"]:
                assert s["ttfc_seconds"] > 0 and 0 <= s["points_before_first"] < s["points_total"]
            else:
                assert s["points_before_first"] == -1
        # plain order: level 1 is pixel-major, so the first counterexample's
        # position is computable from the sorted records
        if ref["cex_total"] and ref["cex_k"][0] == 1:
            assert plain["points_before_first"] == ref["cex_rank"][0]


def test_ranked_search_full_image_matches_oracle(ctx, orc):
    """A 784-pixel property large enough that the ordered search's queue runs
    past its single-chunk tickets into batched ones (4.9 M points, ~77 K
    chunks): both orders return exactly the oracle's records."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(61)
    net = I.random_qnet(g, [784, 64, 64, 10], shift=6, wmax=24, bmax=400)
    m = ibmc.Mlp(ctx, net)
    x = I.workload_blob784(count=1).images[0]
    D = np.array([-32, -16, 16, 32], np.int16)
    ref = orc.q8_check(net, x, D, 1, 2)
    assert ref["cex_total"] > 0
    prop = ibmc.Proposer(ctx, seed=2)
    keys = set(zip(ref["cex_k"].tolist(), ref["cex_rank"].tolist()))
    for p in (None, prop):
        s, cx = ibmc.ibmc_check_property_ranked(ctx, m, p, x, 28, 28, D, 1, 2, cex_capacity=1 << 20)
        assert list(s["cex"]) == [int(v) for v in ref["cex"]]
        assert np.array_equal(cx["rank"], ref["cex_rank"]) and np.array_equal(cx["k"], ref["cex_k"])
        assert np.array_equal(cx["new_label"], ref["cex_label"])
        assert 0 <= s["points_before_first"] < s["points_total"]
        # stopping at the first counterexample still visits every point
        # before it: the same first position, and only true counterexamples
        s1, c1 = ibmc.ibmc_check_property_ranked(ctx, m, p, x, 28, 28, D, 1, 2, stop_at_first=True,
                                                 cex_capacity=1 << 20)
        assert s1["points_before_first"] == s["points_before_first"]
        assert 0 < len(c1) <= len(cx)
        assert all((int(a), int(b)) in keys for a, b in zip(c1["k"], c1["rank"]))


def test_labels_from_records(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(43)
    net = I.random_qnet(g, [30, 64, 16, 5], shift=4, wmax=12, bmax=200)
    m = ibmc.Mlp(ctx, net)
    D = np.array([-48, -16, 16, 48], np.int16)
    x = g.integers(0, 255, size=30, endpoint=True).astype(np.uint8)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
    lab = ibmc.ibmc_label_candidates(ctx, 30, 4, cex)
    exp = np.zeros(30 * 4, np.float32)
    for k, r in zip(cex["k"], cex["rank"]):
        pix, dig = orc.decode(30, 4, int(k), int(r))
        exp[pix * 4 + dig] = 1.0
    assert np.array_equal(lab, exp)
    # counts: the number of records each candidate occurs in
    cnt = ibmc.ibmc_count_candidates(ctx, 30, 4, cex)
    ref = np.zeros(30 * 4, np.float32)
    for k, r in zip(cex["k"], cex["rank"]):
        pix, dig = orc.decode(30, 4, int(k), int(r))
        np.add.at(ref, np.asarray(pix) * 4 + np.asarray(dig), 1.0)
    assert np.array_equal(cnt, ref) and cnt.sum() == int(cex["k"].sum())


def test_fused_scores_match_features_forward(ctx, orc):
    """The one-launch scoring (live norms, features, bf16 MFMA forward) equals
    the network's FP64 forward on the feature rows (themselves pinned to the
    oracle's above), with features and first layer weights rounded to
    bfloat16 as the kernel takes them."""
    from paper_1907_12933_amd import ibmc
    w = I.workload_blob784(count=2)
    m = ibmc.Mlp(ctx, w.net)
    g = I.rng(19)
    prop = ibmc.Proposer(ctx, seed=8)
    W1, b1, w2, c = prop.get()
    prop.set(W1, (g.normal(size=128) * 0.2).astype(np.float32), w2, 0.05)
    W1, b1, w2, c = prop.get()
    for i in range(2):
        f = ibmc.ibmc_proposer_features(ctx, m, w.images[i], 28, 28, w.deltas)
        np.testing.assert_allclose(f, orc.prop_features(w.net, w.images[i], 28, 28, w.deltas), rtol=2e-6, atol=1e-7)
        h = np.maximum(bf16_round(f) @ bf16_round(W1).T + b1.astype(np.float64), 0.0)
        ref = h @ w2.astype(np.float64) + float(c)
        got = ibmc.ibmc_proposer_score(ctx, prop, m, w.images[i], 28, 28, w.deltas).astype(np.float64)
        err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() <= 1e-3, float(err.max())


def _order_keys(scores):
    """16-bit order keys: smaller key = larger score."""
    b = scores.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = np.where(b & 0x80000000, b ^ 0xFFFFFFFF, b | 0x80000000)
    return ((~u) & 0xFFFFFFFF) >> 16


def _order_from_scores(scores):
    """Visiting order of the candidates: 16-bit order keys (larger score first), ties by index."""
    return np.argsort(_order_keys(scores), kind="stable")


def test_ranked_order_follows_scores(ctx, orc):
    """The learned search visits level 1 in score order: its first counterexample's
    position equals the smallest position, in the order computed here from the
    proposer's scores, of the oracle's level-1 counterexamples."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(47)
    net = I.random_qnet(g, [64, 64, 64, 10], shift=5, wmax=16, bmax=200)
    m = ibmc.Mlp(ctx, net)
    D = np.array([-64, -32, 32, 64], np.int16)
    prop = ibmc.Proposer(ctx, seed=2)
    checked = 0
    for t in range(6):
        x = g.integers(0, 255, size=64, endpoint=True).astype(np.uint8)
        ref = orc.q8_check(net, x, D, 1, 1)
        if not ref["cex_total"]:
            continue
        sc = ibmc.ibmc_proposer_score(ctx, prop, m, x, 8, 8, D)
        order = _order_from_scores(sc)
        pos_of = np.empty(len(order), np.int64)
        pos_of[order] = np.arange(len(order))
        expect = min(int(pos_of[int(r)]) for r in ref["cex_rank"])  # k = 1: rank = pixel * m + delta index
        s, _ = ibmc.ibmc_check_property_ranked(ctx, m, prop, x, 8, 8, D, 1, 1)
        assert s["points_before_first"] == expect
        checked += 1
    assert checked >= 2


def test_ranked_order_many_candidates(ctx, orc):
    """12,544 candidates (784 pixels x 16 deltas, many equal 16-bit keys): the
    learned search's first level-1 counterexample sits where the stable order
    of the scores puts the earliest of the oracle's level-1 counterexamples."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(53)
    net = I.random_qnet(g, [784, 64, 16, 10], shift=6, wmax=24, bmax=400)
    m = ibmc.Mlp(ctx, net)
    D = np.array([d for d in range(-64, 65, 8) if d != 0], np.int16)
    assert len(D) == 16
    prop = ibmc.Proposer(ctx, seed=6)
    checked = 0
    for t in range(4):
        x = g.integers(0, 255, size=784, endpoint=True).astype(np.uint8)
        ref = orc.q8_check(net, x, D, 1, 1)
        if not ref["cex_total"]:
            continue
        sc = ibmc.ibmc_proposer_score(ctx, prop, m, x, 28, 28, D)
        order = _order_from_scores(sc)
        key_ties = len(order) - len(np.unique(_order_keys(sc)))
        pos_of = np.empty(len(order), np.int64)
        pos_of[order] = np.arange(len(order))
        expect = min(int(pos_of[int(r)]) for r in ref["cex_rank"])
        s, _ = ibmc.ibmc_check_property_ranked(ctx, m, prop, x, 28, 28, D, 1, 1)
        assert s["points_before_first"] == expect, (t, key_ties)
        checked += 1
    assert checked >= 2


def top_count_labels(counts, frac=0.05):
    """1 for the candidates of one image whose record count lies in the top
    frac of its counts (and is nonzero), else 0."""
    return ((counts >= np.quantile(counts, 1.0 - frac)) & (counts > 0)).astype(np.float32)


def test_trained_proposer_finds_counterexamples_earlier(ctx):
    """Trained on the 64 benchmark images' records (label: the candidate is
    among the 5% taking part in the most counterexamples of its image), the
    proposer's order reaches the first counterexample of held-out images after
    fewer points, at the median, than both the plain order and the same
    network untrained; all three orders return identical records."""
    from paper_1907_12933_amd import ibmc
    w = I.workload_blob784()
    m = ibmc.Mlp(ctx, w.net)
    D = w.deltas
    sums, recs, _, _ = ibmc.ibmc_check_batch(ctx, [(m, x, D, 1, 2) for x in w.images], cex_capacity=1 << 25)
    feats, labels = [], []
    for i, x in enumerate(w.images):
        lo, hi = np.searchsorted(recs["prop"], i, "left"), np.searchsorted(recs["prop"], i, "right")
        assert hi - lo == sums[i]["cex_total"]
        counts = ibmc.ibmc_count_candidates(ctx, 784, len(D), recs[lo:hi])
        feats.append(ibmc.ibmc_proposer_features(ctx, m, x, 28, 28, D))
        labels.append(top_count_labels(counts))
    trained = ibmc.Proposer(ctx, seed=4)
    losses = ibmc.ibmc_proposer_train(ctx, trained, np.concatenate(feats), np.concatenate(labels), epochs=20,
                                      batch=4096, lr=1e-3, seed=4)
    assert losses[-1] < losses[0]
    untrained = ibmc.Proposer(ctx, seed=4)
    pbf = {"plain": [], "untrained": [], "trained": []}
    for x in I.heldout_blob_images():
        out = {}
        for name, p in (("plain", None), ("untrained", untrained), ("trained", trained)):
            out[name] = ibmc.ibmc_check_property_ranked(ctx, m, p, x, 28, 28, D, 1, 2, cex_capacity=1 << 22)
        s0, c0 = out["plain"]
        for name, (s, c) in out.items():
            assert s["cex"] == s0["cex"] and s["clean_label"] == s0["clean_label"]
            assert np.array_equal(c["k"], c0["k"]) and np.array_equal(c["rank"], c0["rank"])
            assert np.array_equal(c["new_label"], c0["new_label"])
        if s0["cex_total"]:
            for name, (s, _) in out.items():
                pbf[name].append(s["points_before_first"])
    assert len(pbf["plain"]) >= 20
    med = {k: float(np.median(v)) for k, v in pbf.items()}
    assert med["trained"] < med["plain"] and med["trained"] < med["untrained"], med
