"""The allocation-free check entry point: same summaries and records as
ibmc_check_property on two calls in a row, the second with a smaller input,
and an oversized request rejected before any device work."""
import numpy as np
import pytest

from paper_1907_12933_amd import ibmc, inputs

pytestmark = pytest.mark.gpu

KEYS = ("clean_label", "first_unsafe_k", "safe_up_to_k", "levels", "points", "cex", "ties", "points_total",
        "cex_total", "near_ties_total", "status")


def _same(got, ref):
    sg, cg, tg = got
    sr, cr, tr = ref
    for key in KEYS:
        assert sg[key] == sr[key], (key, sg[key], sr[key])
    assert np.array_equal(cg, cr) and np.array_equal(tg, tr)


def test_noalloc_matches_check_property_on_two_calls():
    ctx = ibmc.Context(0)
    # call 1: blob image 0 of the 784-256-256-10 net, k = 1..2 (11,054,400
    # points, 176,982 counterexamples by the oracle)
    w = inputs.workload_blob784(count=1)
    big = ibmc.Mlp(ctx, w.net)
    print("noalloc call 1: blob784 image 0, k=1..2", flush=True)
    got = ibmc.ibmc_check_property_noalloc(ctx, big, w.images[0], w.deltas, 1, 2, cex_capacity=1 << 18)
    ref = ibmc.ibmc_check_property(ctx, big, w.images[0], w.deltas, 1, 2, cex_capacity=1 << 18)
    assert ref[0]["cex_total"] == 176982
    _same(got, ref)
    # call 2, smaller: a 24-64-16-5 net (shift 4), four deltas, k = 1..2
    g = inputs.rng(7)
    net = inputs.random_qnet(g, [24, 64, 16, 5], shift=4, wmax=12, bmax=100)
    x = g.integers(0, 255, size=24, endpoint=True).astype(np.uint8)
    D = np.array([-96, -48, 48, 96], np.int16)
    small = ibmc.Mlp(ctx, net)
    print("noalloc call 2: 24-64-16-5, k=1..2", flush=True)
    got = ibmc.ibmc_check_property_noalloc(ctx, small, x, D, 1, 2, cex_capacity=1 << 10)
    ref = ibmc.ibmc_check_property(ctx, small, x, D, 1, 2, cex_capacity=1 << 10)
    assert ref[0]["cex_total"] > 0
    _same(got, ref)
    # a capacity whose record space exceeds the fixed scratch is refused
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_check_property_noalloc(ctx, big, w.images[0], w.deltas, 1, 2, cex_capacity=1 << 22)
    assert e.value.code == ibmc.IBMC_E_INVALID and "fixed scratch" in str(e.value)
