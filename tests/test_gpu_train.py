"""GPU parity of the training of the float networks (trained on labelled
examples, Sec. II-A) and of the counterexample-augmented retraining loop
(the verifier's counterexamples added to the training set, Sec. VI):

  - the loss and gradient of labelled sets against the oracle's FP64
    backpropagation, on networks of two to four layers, a 1024-wide one
    whose samples span several launches, a single sample and ragged tiles;
  - mini-batch Adam against the oracle's FP64 Adam on the same sample order
    (ragged last batch), and the library's own shuffle run twice;
  - the loop: train on a labelled glyph set, check robustness properties,
    add every counterexample with its clean image's label, retrain, check
    again: fewer counterexamples, and the re-check of the retrained network
    equal to the oracle's FP64 check of the same weights.

Tolerances: the kernels accumulate in FP32 (dot products of at most 1,024
terms, sums over at most 16 samples per workgroup and then over
workgroups); each sum's rounding is within K 2^-24 of the sum of absolute
terms (K terms), so the gradient is compared within 2e-4 of its largest
entry and the loss within 1e-5 relative."""
import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def flat(W, b):
    return np.concatenate([np.concatenate([np.asarray(w, np.float64).reshape(-1), np.asarray(x, np.float64)])
                           for w, x in zip(W, b)])


@pytest.mark.parametrize("dims,n,seed", [([35, 16, 5], 37, 1), ([49, 128, 64, 10], 100, 2), ([12, 16, 8, 4], 1, 3),
                                         ([30, 200, 100, 50, 10], 53, 4), ([20, 1024, 10], 9, 5),
                                         ([784, 1024, 1024, 1024, 10], 100, 6)])
def test_loss_grad_matches_oracle(ctx, orc, dims, n, seed):
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.random_fnet(g, dims, scale=2.0)
    net.b = [(g.standard_normal(d) * 0.5).astype(np.float32) for d in dims[1:]]
    imgs = g.integers(0, 255, size=(n, dims[0]), endpoint=True).astype(np.uint8)
    labs = g.integers(0, dims[-1] - 1, size=n, endpoint=True).astype(np.int32)
    m = ibmc.Mlp(ctx, net)
    loss, grad = ibmc.ibmc_mlp_loss_grad(ctx, m, imgs, labs)
    rl, rg = orc.f64_loss_grad(net, imgs, labs)
    print(f"{dims} n={n}: loss {loss:.6f} vs {rl:.6f}, max grad err {np.max(np.abs(grad - rg)):.3e} "
          f"of max {np.max(np.abs(rg)):.3e}")
    assert loss == pytest.approx(rl, rel=1e-5)
    assert np.max(np.abs(grad - rg)) <= 2e-4 * np.max(np.abs(rg))


def test_fit_matches_oracle_adam(ctx, orc):
    from paper_1907_12933_amd import ibmc
    g = I.rng(21)
    _, X, Y = I.labelled_glyphs(g, 5, 50, proto_flip=0.2)
    net = I.random_fnet(g, [35, 16, 5])
    order = np.stack([g.permutation(50) for _ in range(3)])
    m = ibmc.Mlp(ctx, net)
    m1, losses = ibmc.ibmc_fit_mlp(ctx, m, X, Y, epochs=3, batch=8, lr=1e-2, order=order)
    W, b, rl = orc.f64_fit(net, X, Y, order, batch=8, lr=1e-2)
    got, ref = flat(*m1.params), flat(W, b)
    print(f"theta max diff {np.max(np.abs(got - ref)):.3e}, losses {losses} vs {rl}")
    # 21 Adam steps of at most lr each per parameter
    assert np.max(np.abs(got - ref)) <= 1e-4 * 21 * 1e-2
    assert np.allclose(losses, rl, rtol=1e-5)
    assert losses[-1] < losses[0]
    # the source network is unchanged and the trained one loads as a network
    assert np.array_equal(flat(*m.params), flat(net.W, net.b))
    l1, _ = ibmc.ibmc_mlp_loss_grad(ctx, m1, X, Y)
    assert l1 == pytest.approx(orc.f64_loss_grad(I.FNet(net.dims, *m1.params), X, Y)[0], rel=1e-5)


def test_fit_own_shuffle_is_reproducible(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(22)
    _, X, Y = I.labelled_glyphs(g, 4, 70)
    m = ibmc.Mlp(ctx, I.random_fnet(g, [35, 24, 4]))
    a, la = ibmc.ibmc_fit_mlp(ctx, m, X, Y, epochs=4, batch=16, lr=5e-3, seed=7)
    b, lb = ibmc.ibmc_fit_mlp(ctx, m, X, Y, epochs=4, batch=16, lr=5e-3, seed=7)
    c, _ = ibmc.ibmc_fit_mlp(ctx, m, X, Y, epochs=4, batch=16, lr=5e-3, seed=8)
    assert np.array_equal(flat(*a.params), flat(*b.params)) and np.array_equal(la, lb)
    assert not np.array_equal(flat(*a.params), flat(*c.params))


def perturbed(x, D, pix, dig):
    xp = x.astype(np.int64).copy()
    for p, d in zip(pix, dig):
        xp[p] = min(255, max(0, xp[p] + int(D[d])))
    return xp.astype(np.uint8)


def test_retraining_on_counterexamples(ctx, orc):
    """Train, check, add the counterexamples with their clean labels,
    retrain, check again."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(13)
    _, X, Y = I.labelled_glyphs(g, 10, 400, p_flip=0.03, proto_flip=0.15)
    net = I.random_fnet(g, [35, 16, 10])
    m0, l0 = ibmc.ibmc_fit_mlp(ctx, ibmc.Mlp(ctx, net), X, Y, epochs=40, batch=32, lr=1e-2, seed=1)
    assert l0[-1] < 0.1 * l0[0]
    D = np.array([-255, 255], np.int16)
    props = range(12)

    def check(mm):
        out = []
        for i in props:
            s, cex, ties = ibmc.ibmc_check_property(ctx, mm, X[i], D, 1, 2, near_tie_capacity=1 << 16)
            out.append((i, cex, ties))
        return out

    before = check(m0)
    n0 = sum(len(c) for _, c, _ in before)
    aug_x, aug_y = [], []
    for i, cex, _ in before:
        for k, r in zip(cex["k"], cex["rank"]):
            pix, dig = ibmc.ibmc_decode_point(35, len(D), int(k), int(r))
            aug_x.append(perturbed(X[i], D, pix, dig))
            aug_y.append(Y[i])
    assert n0 > 50
    X2 = np.concatenate([X, np.stack(aug_x)])
    Y2 = np.concatenate([Y, np.array(aug_y, np.int32)])
    m1, l1 = ibmc.ibmc_fit_mlp(ctx, m0, X2, Y2, epochs=20, batch=32, lr=5e-3, seed=2)
    after = check(m1)
    n1 = sum(len(c) for _, c, _ in after)
    print(f"counterexamples on 12 properties: {n0} before, {n1} after retraining on {len(aug_x)} of them")
    assert n1 < n0 / 2
    # the re-check equals the oracle's FP64 check of the retrained weights
    net1 = I.FNet(net.dims, *m1.params)
    for i, cex, ties in after:
        r = orc.f64_check(net1, X[i], D, 1, 2, tie_rel=0.0)
        got = set(zip(cex["k"].tolist(), cex["rank"].tolist()))
        ref = set(zip(r["cex_k"].tolist(), r["cex_rank"].tolist()))
        assert got ^ ref <= set(zip(ties["k"].tolist(), ties["rank"].tolist()))


def test_train_refusals(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(23)
    q = ibmc.Mlp(ctx, I.random_qnet(g, [20, 16, 5], shift=6))
    f = ibmc.Mlp(ctx, I.random_fnet(g, [20, 16, 5]))
    x = g.integers(0, 255, size=(4, 20), endpoint=True).astype(np.uint8)
    y = np.array([0, 1, 2, 3], np.int32)
    cases = [(lambda: ibmc.ibmc_mlp_loss_grad(ctx, q, x, y), ibmc.IBMC_E_UNIMPL),
             (lambda: ibmc.ibmc_fit_mlp(ctx, q, x, y), ibmc.IBMC_E_UNIMPL),
             (lambda: ibmc.ibmc_mlp_loss_grad(ctx, f, x, np.array([0, 1, 2, 5], np.int32)), ibmc.IBMC_E_INVALID),
             (lambda: ibmc.ibmc_fit_mlp(ctx, f, x, y, epochs=0), ibmc.IBMC_E_INVALID),
             (lambda: ibmc.ibmc_fit_mlp(ctx, f, x, y, lr=0.0), ibmc.IBMC_E_INVALID),
             (lambda: ibmc.ibmc_fit_mlp(ctx, f, x, y, epochs=1, order=np.array([[0, 1, 2, 4]])), ibmc.IBMC_E_INVALID)]
    for fn, code in cases:
        with pytest.raises(ibmc.IbmcError) as e:
            fn()
        assert e.value.code == code


def test_fit_wide_net_split_batches_matches_oracle(ctx, orc):
    """A batch whose partial rows exceed one launch's budget (784-1024-1024-
    1024-10, 2.9 M parameters: the gradient is accumulated over several
    launches before the Adam step) against the oracle's FP64 Adam."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(24)
    dims = [784, 1024, 1024, 1024, 10]
    net = I.random_fnet(g, dims)
    X = g.integers(0, 255, size=(70, 784), endpoint=True).astype(np.uint8)
    Y = g.integers(0, 9, size=70, endpoint=True).astype(np.int32)
    order = np.stack([g.permutation(70)])
    m1, losses = ibmc.ibmc_fit_mlp(ctx, ibmc.Mlp(ctx, net), X, Y, epochs=1, batch=64, lr=1e-3, order=order)
    W, b, rl = orc.f64_fit(net, X, Y, order, batch=64, lr=1e-3)
    got, ref = flat(*m1.params), flat(W, b)
    # Adam moves a parameter by about lr whatever its gradient's size, so a
    # gradient within the FP32 rounding of zero may step either way: the
    # strict bound holds where the first batch's gradient is clear of it
    _, g0 = orc.f64_loss_grad(net, X[order[0][:64]], Y[order[0][:64]])
    clear = np.abs(g0) > 1e-3 * np.max(np.abs(g0))
    d = np.abs(got - ref)
    print(f"wide fit: theta max diff {d[clear].max():.3e} where the gradient is clear of zero "
          f"({clear.mean():.4f} of the parameters), {d.max():.3e} overall; losses {losses} vs {rl}")
    assert d[clear].max() <= 1e-4 * 2 * 1e-3
    assert d.max() <= 2 * 2 * 1e-3
    assert np.allclose(losses, rl, rtol=1e-5)
