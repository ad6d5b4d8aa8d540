"""Boundary entry points and robustness of the check (C ABI through ctypes):
resumable checks (chunk budget and resume cursor), an abort from another
host thread, device-pointer variants, and the increment granularity k_step
of the incremental bound (Sec. II-B)."""
import threading
import time

import numpy as np
import pytest

from paper_1907_12933_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1907_12933_amd import ibmc
    return ibmc.Context(0)


def keyset(recs):
    return set(zip(recs["prop"].tolist(), recs["k"].tolist(), recs["rank"].tolist(), recs["new_label"].tolist()))


def test_budgeted_calls_resume_to_the_full_check(ctx):
    """A check cut into budgeted calls, each resumed from the previous call's
    next_cursor, returns exactly the records and counts of one call."""
    from paper_1907_12933_amd import ibmc
    w = I.workload_blob784(count=1)
    m = ibmc.Mlp(ctx, w.net)
    full, fcex, _ = ibmc.ibmc_check_property(ctx, m, w.images[0], w.deltas, 1, 2, cex_capacity=1 << 18)
    assert full["next_cursor"] == -1 and full["cex_total"] == 176982
    cursor, parts, calls = 0, [], 0
    cex_sum = np.zeros(2, np.int64)
    ties_sum = np.zeros(2, np.int64)
    while True:
        s, cex, _ = ibmc.ibmc_check_property(ctx, m, w.images[0], w.deltas, 1, 2, cex_capacity=1 << 18,
                                             resume_cursor=cursor, chunk_budget=15000)
        calls += 1
        parts.append(cex)
        cex_sum += s["cex"]
        ties_sum += s["ties"]
        if s["next_cursor"] < 0:
            assert s["status"] == ibmc.IBMC_OK
            break
        assert s["status"] == ibmc.IBMC_W_PARTIAL and s["next_cursor"] > cursor
        cursor = s["next_cursor"]
        assert calls < 100
    assert calls >= 3
    assert list(cex_sum) == full["cex"] and list(ties_sum) == full["ties"]
    allp = np.concatenate(parts)
    assert len(allp) == len(fcex) and keyset(allp) == keyset(fcex)


def test_resume_is_refused_where_undefined(ctx):
    from paper_1907_12933_amd import ibmc
    g = I.rng(5)
    q = I.random_qnet(g, [20, 64, 16, 5], shift=5)
    x = g.integers(0, 255, size=20, endpoint=True).astype(np.uint8)
    D = np.array([-40, 40], np.int16)
    fm = ibmc.Mlp(ctx, I.fnet_from_qnet(q))
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_check_property(ctx, fm, x, D, 1, 2, chunk_budget=10)
    assert e.value.code == ibmc.IBMC_E_UNIMPL
    qm = ibmc.Mlp(ctx, q)
    with pytest.raises(ibmc.IbmcError) as e:
        ibmc.ibmc_check_property(ctx, qm, x, D, 1, 2, chunk_budget=10, stop_at_first=True)
    assert e.value.code == ibmc.IBMC_E_UNIMPL


def test_abort_from_another_thread(ctx):
    """ibmc_abort from a host thread while the 64-image check runs: the
    kernel gives up through its own poll, the call returns IBMC_E_ABORTED
    early with the counts and records of the chunks it finished (all true
    counterexamples), and resuming from its next_cursor completes the check."""
    import torch
    from paper_1907_12933_amd import ibmc
    w = I.workload_blob784()
    m = ibmc.Mlp(ctx, w.net)
    imgs = torch.from_numpy(w.images).cuda()
    props = [(m, imgs[i], w.deltas, 1, 2) for i in range(len(w.images))]
    t0 = time.perf_counter()
    full, fcex, _, rc = ibmc.ibmc_check_batch_dev(ctx, props, cex_capacity=1 << 25)
    t_full = time.perf_counter() - t0
    assert rc == ibmc.IBMC_OK and full[0]["next_cursor"] == -1
    fkeys = keyset(fcex)
    for attempt in range(3):
        timer = threading.Timer(0.25 * t_full, ibmc.ibmc_abort, args=(ctx,))
        t0 = time.perf_counter()
        timer.start()
        sums, pcex, _, rc = ibmc.ibmc_check_batch_dev(ctx, props, cex_capacity=1 << 25, allow_abort=True)
        t_part = time.perf_counter() - t0
        timer.join()
        if rc == ibmc.IBMC_E_ABORTED:
            break
    assert rc == ibmc.IBMC_E_ABORTED, "the abort never landed inside the call"
    assert t_part < 0.9 * t_full + 0.05
    cursor = sums[0]["next_cursor"]
    assert cursor > 0
    pkeys = keyset(pcex)
    assert len(pkeys) == len(pcex) < len(fcex)
    assert pkeys <= fkeys                          # only true counterexamples
    for s, f in zip(sums, full):
        assert all(a <= b for a, b in zip(s["cex"], f["cex"]))
    # resuming from the cursor finishes the check: the union is the full list
    rest, rcex, _, rc2 = ibmc.ibmc_check_batch_dev(ctx, props, cex_capacity=1 << 25, resume_cursor=cursor)
    assert rc2 == ibmc.IBMC_OK and rest[0]["next_cursor"] == -1
    assert len(pcex) + len(rcex) == len(fcex)
    assert pkeys | keyset(rcex) == fkeys
    for a, b, f in zip(sums, rest, full):
        assert [x + y for x, y in zip(a["cex"], b["cex"])] == f["cex"]


def test_device_image_variants(ctx, orc):
    import torch
    from paper_1907_12933_amd import ibmc
    g = I.rng(42)
    net = I.random_qnet(g, [48, 64, 32, 6], shift=12, wmax=127, bmax=1 << 16)
    net.shift = [11, 9]
    x = g.integers(0, 255, size=48, endpoint=True).astype(np.uint8)
    D = np.array([-255, -128, 128, 255], np.int16)
    m = ibmc.Mlp(ctx, net)
    s1, c1, _ = ibmc.ibmc_check_property(ctx, m, x, D, 1, 2)
    s2, c2, _ = ibmc.ibmc_check_property_dev(ctx, m, torch.from_numpy(x).cuda(), D, 1, 2)
    assert s1["cex"] == s2["cex"] and np.array_equal(c1, c2) and s1["cex_total"] > 0
    # proposer scores from a device image into a device buffer
    w = I.workload_blob784(count=1)
    bm = ibmc.Mlp(ctx, w.net)
    prop = ibmc.Proposer(ctx, seed=3)
    host = ibmc.ibmc_proposer_score(ctx, prop, bm, w.images[0], 28, 28, w.deltas)
    dev = torch.empty(784 * len(w.deltas), dtype=torch.float32, device="cuda")
    ibmc.ibmc_proposer_score_dev(ctx, prop, bm, torch.from_numpy(w.images[0]).cuda(), 28, 28, w.deltas, dev)
    assert np.array_equal(dev.cpu().numpy(), host)


@pytest.mark.parametrize("seed,dims,kmin,kmax", [(60, [12, 64, 16, 4], 1, 5), (60, [10, 64, 8], 0, 4)])
def test_k_step_two(ctx, orc, seed, dims, kmin, kmax):
    """Increment granularity 2: levels k_min, k_min + 2, ... only, each equal
    to the oracle's."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(seed)
    net = I.random_qnet(g, dims, shift=5, wmax=40, bmax=300)
    x = g.integers(0, 255, size=dims[0], endpoint=True).astype(np.uint8)
    D = np.array([-90, -30, 30, 90], np.int16)
    m = ibmc.Mlp(ctx, net)
    s, cex, _ = ibmc.ibmc_check_property(ctx, m, x, D, kmin, kmax, k_step=2, cex_capacity=1 << 22)
    r = orc.q8_check(net, x, D, kmin, kmax, k_step=2, cap=1 << 22)
    assert s["levels"] == list(range(kmin, kmax + 1, 2)) == list(r["levels"])
    assert s["cex"] == [int(v) for v in r["cex"]] and s["ties"] == [int(v) for v in r["ties"]]
    assert np.array_equal(cex["k"], r["cex_k"]) and np.array_equal(cex["rank"], r["cex_rank"])
    assert np.array_equal(cex["new_label"], r["cex_label"])
    assert r["cex_total"] > 0


def test_network_outlives_its_context():
    """A network freed after its context (the order a garbage collector may
    pick) leaves no error behind for the next context's calls."""
    from paper_1907_12933_amd import ibmc
    g = I.rng(9)
    net = I.random_qnet(g, [20, 16, 5], shift=5)
    c = ibmc.Context(0)
    m = ibmc.Mlp(c, net)
    c.close()
    m.close()
    c2 = ibmc.Context(0)
    m2 = ibmc.Mlp(c2, net)
    x = g.integers(0, 255, size=20, endpoint=True).astype(np.uint8)
    s, _, _ = ibmc.ibmc_check_property(c2, m2, x, np.array([-40, 40], np.int16), 1, 2)
    assert s["points_total"] == 20 * 2 + 190 * 4
