"""Throughput of the exhaustive check on one MI355X.

Workload (one step): the 784-256-256-10 int8 network on 64 synthetic 28x28
blob images, every point with k = 1 and k = 2 changed pixels and deltas in
{+-8, +-16, +-32} (11,054,400 points per image, 707,481,600 per step), all
counterexamples returned to the host.  Images are resident in device memory
before the timed region.  Prints one JSON line.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

MI355X_INT8_PEAK_TOPS = 5000.0     # dense int8 MFMA, TOP/s
MI355X_FP32_PEAK_TFLOPS = 157.3    # FP32 vector, TFLOP/s (half of it without packed FP32)
MI355X_HBM_PEAK_GBS = 8000.0
MI355X_SPEC_CLOCK_GHZ = 2.4
HERE = os.path.dirname(os.path.abspath(__file__))
# enumeration kernel sources whose hash keys the profile record
TUNE_TABLE = os.path.join(HERE, "paper_1907_12933_amd", "tune_gfx950.json")
KERNEL_SOURCES = ["paper_1907_12933_amd/csrc/enum_q8_impl.h", "paper_1907_12933_amd/csrc/enum_common.h",
                  "paper_1907_12933_amd/csrc/ibmc_internal.h"]


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_record():
    """The rocprofv3 figures of the enumeration kernel on this workload kept in
    profiles/ (kernel-trace average duration of this benchmark's command, HBM
    bytes per launch from FETCH_SIZE / WRITE_SIZE scaled by a plain copy's
    counters, shader clock and matrix-pipe busy from the counter run), or None
    once the kernel sources differ from the ones profiled."""
    path = os.path.join(HERE, "profiles", "enum_q8_blob784.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec if rec.get("kernel_source_sha256") == kernel_source_sha() else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(O, w, threads, target_seconds, seed):
    """Points/s of the oracle on a seeded random sample of the workload's
    points (image 0, levels 1 and 2 in proportion), grown until about
    target_seconds of work."""
    n, m = w.net.dims[0], len(w.deltas)
    n1, n2 = O.points(n, m, 1), O.points(n, m, 2)
    g = np.random.Generator(np.random.PCG64(seed))
    size = 2000 if threads == 1 else 20000
    total_pts, total_t = 0, 0.0
    while total_t < target_seconds:
        ks = np.where(g.random(size) < n1 / (n1 + n2), 1, 2).astype(np.int32)
        ranks = np.where(ks == 1, g.integers(0, n1, size), g.integers(0, n2, size)).astype(np.int64)
        t0 = time.perf_counter()
        O.q8_eval_points(w.net, w.images[0], w.deltas, ks, ranks, nthreads=threads)
        dt = time.perf_counter() - t0
        total_pts += size
        total_t += dt
        size = int(min(max(size * 2, 1), max(1, (target_seconds - total_t) / max(dt / size, 1e-9))) + 1)
        if target_seconds - total_t < 0.5:
            break
    return total_pts / total_t, total_pts, total_t


def cpu_baseline(w, target_seconds=15.0):
    """The oracle (plain full int64 forward per point) on a bounded sample of
    the same workload, on all host cores and on one core."""
    from oracle import oracle as O
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    rate, pts, t = _oracle_rate(O, w, threads, target_seconds, 1234)
    rate1, pts1, t1 = _oracle_rate(O, w, 1, 5.0, 4321)
    return dict(value=rate, unit="points/s", cores=threads, kind="oracle",
                sample=f"{pts} seeded random points (k=1 and k=2 in proportion) of image 0, "
                       f"full int64 forward per point, {t:.1f} s",
                single_core_value=rate1, single_core_sample=f"{pts1} points, {t1:.1f} s",
                cpu_model=cpu_model())


def top_count_labels(counts, frac=0.05):
    """1 for the candidates of one image whose record count lies in the top
    frac of its counts (and is nonzero), else 0."""
    return ((counts >= np.quantile(counts, 1.0 - frac)) & (counts > 0)).astype(np.float32)


def proposer_leg(ctx, ibmc, inputs, w, net, recs, args):
    """Train the proposal network on the step's 64 blob images (label: the
    candidate is among the 5% of its image taking part in the most
    counterexamples), then search 64 held-out blob images in plain order,
    untrained-proposer order and trained-proposer order: points visited and
    host time before the first counterexample; every held-out verdict and
    record list must be identical across the three."""
    t_all = time.perf_counter()
    feats, labels = [], []
    props_col = recs["prop"]
    for i in range(len(w.images)):
        lo, hi = np.searchsorted(props_col, i, "left"), np.searchsorted(props_col, i, "right")
        counts = ibmc.ibmc_count_candidates(ctx, 784, len(w.deltas), recs[lo:hi])
        labels.append(top_count_labels(counts))
        feats.append(ibmc.ibmc_proposer_features(ctx, net, w.images[i], 28, 28, w.deltas))
    F = np.concatenate(feats)
    Y = np.concatenate(labels)
    prop = ibmc.Proposer(ctx, seed=4)
    t0 = time.perf_counter()
    losses = ibmc.ibmc_proposer_train(ctx, prop, F, Y, epochs=20, batch=4096, lr=1e-3, seed=4)
    t_train = time.perf_counter() - t0
    untrained = ibmc.Proposer(ctx, seed=4)
    held = inputs.heldout_blob_images()
    orders = (("plain", None), ("untrained", untrained), ("trained", prop))
    rows = []
    identical = True
    for x in held:
        res = {}
        for name, p in orders:
            res[name] = ibmc.ibmc_check_property_ranked(ctx, net, p, x, 28, 28, w.deltas, 1, 2, cex_capacity=1 << 22)
        s0, c0 = res["plain"]
        for name, (s, c) in res.items():
            identical &= (s["cex"] == s0["cex"] and s["clean_label"] == s0["clean_label"]
                          and np.array_equal(c["rank"], c0["rank"]) and np.array_equal(c["k"], c0["k"]))
        if s0["cex_total"] > 0:
            rows.append({name: (s["points_before_first"], s["ttfc_seconds"]) for name, (s, _) in res.items()})
    med = lambda v: float(np.median(v)) if len(v) else None
    out = dict(
        labels="top 5% of candidates by record count per image", train_images=len(w.images),
        train_samples=int(len(Y)), train_positive=int(Y.sum()), epochs=20, batch=4096,
        loss_first=float(losses[0]), loss_last=float(losses[-1]), train_seconds=round(t_train, 3),
        heldout_images=len(held), heldout_unsafe=len(rows), identical_verdicts=bool(identical))
    n_cu = ctx.device_info()[0]
    # the first round of the persistent grid (two workgroups of four waves
    # per compute unit, one 64-point chunk each) is visited at once, so the
    # order only decides the time of first hits that lie beyond it
    round_pts = n_cu * 2 * 4 * 64
    out["first_round_points"] = int(round_pts)
    late = [r for r in rows if r["plain"][0] >= round_pts]
    out["late_images"] = len(late)
    for name, _ in orders:
        pb = [r[name][0] for r in rows]
        tt = [r[name][1] for r in rows]
        out[name] = dict(
            points_before_first_median=med(pb), points_before_first_total=int(sum(pb)),
            ttfc_median_s=med(tt), ttfc_mean_s=float(np.mean(tt)) if tt else None,
            ttfc_total_s=float(sum(tt)),
            ttfc_late_median_s=med([r[name][1] for r in late]),
            first_before_plain=int(sum(1 for r in rows if r[name][0] < r["plain"][0])))
    out["leg_seconds"] = round(time.perf_counter() - t_all, 2)
    return out


def coverage_leg(ctx, ibmc, inputs, torch):
    """SS/DS/SV/DV over 4,096 pairs of the 784-1024-1024-1024-10 net, and the
    same sweep over 65,536 pairs.  Algorithmic work per pair: x1's full
    forward plus x2's layers >= 2 and its first layer as the rank-r update
    (r changed pixels times the first hidden width), 2 ops per MAC."""
    out = {}
    for n_pairs in (4096, 65536):
        net, x1, x2 = inputs.coverage_pairs_blob784(n_pairs=n_pairs)
        m = ibmc.Mlp(ctx, net)
        d1, d2 = torch.from_numpy(x1).cuda(), torch.from_numpy(x2).cuda()
        ibmc.ibmc_coverage_all_dev(ctx, m, d1, d2, want_bits=False)
        ts, dev = [], []
        for _ in range(5):
            t0 = time.perf_counter()
            res = ibmc.ibmc_coverage_all_dev(ctx, m, d1, d2, want_bits=False)
            ts.append(time.perf_counter() - t0)
            dev.append(res[0]["seconds"])
        dims = net.dims
        full = sum(dims[l] * dims[l + 1] for l in range(len(dims) - 1))
        r = int(np.count_nonzero(x1 != x2))
        macs = n_pairs * (2 * full - dims[0] * dims[1]) + r * dims[1]
        t, td = float(np.median(ts)), float(np.median(dev))
        out[f"pairs_{n_pairs}"] = dict(
            seconds=round(t, 6), device_seconds=round(td, 6), int8_macs=macs, changed_pixels=r,
            int8_tops=round(2 * macs / td / 1e12, 2), frac_int8_peak=round(2 * macs / td / 5e15, 4),
            criteria={c: dict(covered_pairs=q["covered_pairs"], total_pairs=q["total_pairs"],
                              covered_neurons=q["covered_neurons"], total_neurons=q["total_neurons"],
                              fraction=round(q["fraction"], 4), literal=q["literal"])
                      for c, q in zip(["SS", "DS", "SV", "DV"], res)})
    out["workload"] = "784-1024-1024-1024-10, pairs differing in 1-8 pixels (4,096 and 65,536 pairs), all four criteria"
    return out


def dense_macs(dims):
    """int8 MACs of the dense layers >= 2 (the first layer is the rank-k update)."""
    return sum(dims[l] * dims[l + 1] for l in range(1, len(dims) - 1))


def f32_flops(dims):
    """Algorithmic FP32 operations of one point of the float variant: the
    first-layer update (one FMA per unit), the later layers' FMAs, and four
    operations per sigmoid (scale, exponential, add, reciprocal)."""
    fma = dims[1] + dense_macs(dims)
    return 2 * fma + 4 * sum(dims[1:-1])


def batch_leg(ctx, ibmc, inputs):
    """256 properties over eight uneven nets (k <= 3, per-property deltas) as one
    graph of persistent launches; and 64 FP32-sigmoid properties."""
    nets, props = inputs.batch_workload(seed=3)
    ms = [ibmc.Mlp(ctx, n) for n in nets]
    P = [(ms[p.net_index], p.image, p.deltas, 1, p.k) for p in props]
    ibmc.ibmc_check_batch(ctx, P, cex_capacity=1 << 24)
    t0 = time.perf_counter()
    sums, cex, _, rc = ibmc.ibmc_check_batch(ctx, P, cex_capacity=1 << 24)
    t = time.perf_counter() - t0
    dev = sums[0]["seconds"]
    pts = sum(s["points_total"] for s in sums)
    # point-weighted int8 work of the batch: each property's points times its
    # network's dense later-layer MACs
    ops = sum(2.0 * s["points_total"] * dense_macs(nets[p.net_index].dims) for s, p in zip(sums, props))
    fn, fp = inputs.batch_workload(seed=33, per_net=8, mac_budget=2e11)
    fms = [ibmc.Mlp(ctx, inputs.fnet_from_qnet(n)) for n in fn]
    FP = [(fms[p.net_index], p.image, p.deltas, 1, p.k) for p in fp]
    ibmc.ibmc_check_batch(ctx, FP, cex_capacity=1 << 22, near_tie_capacity=1 << 20)
    t1 = time.perf_counter()
    fs, fc, ft, _ = ibmc.ibmc_check_batch(ctx, FP, cex_capacity=1 << 22, near_tie_capacity=1 << 20)
    tf = time.perf_counter() - t1
    fdev = fs[0]["seconds"]
    fpts = sum(s["points_total"] for s in fs)
    fflops = sum(float(s["points_total"]) * f32_flops(fn[p.net_index].dims) for s, p in zip(fs, fp))
    launches, replays = ibmc.ibmc_graph_stats(ctx)
    return dict(properties=len(props), networks=len(nets), points=pts, seconds=round(t, 4),
                device_seconds=round(dev, 4), points_per_s=pts / t,
                kernels={"_".join(map(str, n.dims)): ibmc.ibmc_chosen_variant(ctx, m) for n, m in zip(nets, ms)},
                graph_launches=launches, graph_replays=replays,
                counterexamples=int(sum(s["cex_total"] for s in sums)),
                int8_roofline=dict(bound="mfma", achieved=round(ops / dev / 1e12, 2), peak=MI355X_INT8_PEAK_TOPS,
                                   unit="TOP/s", frac=round(ops / dev / 1e12 / MI355X_INT8_PEAK_TOPS, 4),
                                   work="sum over properties of points x dense later-layer MACs x 2, "
                                        "over the batch call's device time"),
                fp32_properties=len(fp), fp32_points=fpts, fp32_seconds=round(tf, 4),
                fp32_device_seconds=round(fdev, 4), fp32_points_per_s=fpts / tf,
                fp32_near_ties=int(sum(s["near_ties_total"] for s in fs)),
                fp32_roofline=dict(bound="alu", achieved=round(fflops / fdev / 1e12, 2),
                                   peak=MI355X_FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                   frac=round(fflops / fdev / 1e12 / MI355X_FP32_PEAK_TFLOPS, 4),
                                   work="per point 2 x (first-layer update + later-layer FMAs) + 4 per sigmoid, "
                                        "over the batch call's device time"))


def glyph_leg(ctx, ibmc, inputs):
    """The CPU-sized plain workload: 35-16-5 net, ten 7x5 glyphs, deltas
    -16..16, k <= 2 (649,110 points per image), as one batch."""
    g = inputs.workload_glyph35()
    m = ibmc.Mlp(ctx, g.net)
    P = [(m, x, g.deltas, 1, 2) for x in g.images]
    ibmc.ibmc_check_batch(ctx, P, cex_capacity=1 << 20)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        sums, _, _, _ = ibmc.ibmc_check_batch(ctx, P, cex_capacity=1 << 20)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    pts = sum(s["points_total"] for s in sums)
    return dict(workload="glyph35: 35-16-5, 10 glyph images, deltas -16..16, k=1..2", points=pts,
                seconds=round(t, 6), points_per_s=pts / t, us_per_image=round(t / len(P) * 1e6, 2),
                counterexamples=int(sum(s["cex_total"] for s in sums)))


def covsearch_leg(ctx, ibmc, inputs):
    """Coverage-guided test generation (the covers of Sec. III-B as the
    objective, Sec. IV-C): a seeded 30-40-30-6 integer net (shifts 5 and 4)
    and a random 30-pixel image; every point of level 2 of the deltas
    +-20/+-60/+-120 (15,660 candidate tests) scored for each criterion, and up
    to 64 tests taken greedily."""
    g = inputs.rng(33)
    net = inputs.random_qnet(g, [30, 40, 30, 6], shift=[5, 4], wmax=40, bmax=300)
    x = g.integers(0, 255, size=30, endpoint=True).astype(np.uint8)
    D = np.array([-120, -60, -20, 20, 60, 120], np.int16)
    m = ibmc.Mlp(ctx, net)
    out = {}
    for crit in ("SS", "DS", "SV", "DV"):
        ibmc.ibmc_coverage_search(ctx, m, x, D, 2, crit, max_tests=64)
        t0 = time.perf_counter()
        tests, gains, cov = ibmc.ibmc_coverage_search(ctx, m, x, D, 2, crit, max_tests=64)
        t = time.perf_counter() - t0
        out[crit] = dict(seconds=round(t, 5), tests=len(tests), covered_pairs=cov["covered_pairs"],
                         total_pairs=cov["total_pairs"], first_gain=int(gains[0]) if len(gains) else 0,
                         candidates_per_s=round(435 * 36 / t))
    out["workload"] = "30-40-30-6 net (seed 33), one random image, level k = 2 of 6 deltas (15,660 candidate tests)"
    return out


def ball_leg(ctx, ibmc, inputs):
    """The paper's own domain (Sec. III-C, Eq. (9)): every image within L2
    distance gamma * 255 of each of the ten 7x5 glyphs of the 35-16-5 net,
    levels k = 1, 2 by support size, for the two smallest proximities of
    Table III (gamma = 0.3 and 0.5), as one batch per radius."""
    g = inputs.workload_glyph35()
    m = ibmc.Mlp(ctx, g.net)
    out = {}
    for gamma in (0.3, 0.5):
        r2 = int((gamma * 255) ** 2)
        P = [(m, x, r2, 1, 2) for x in g.images]
        ibmc.ibmc_check_ball_batch(ctx, P, cex_capacity=1 << 22)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            sums, cex = ibmc.ibmc_check_ball_batch(ctx, P, cex_capacity=1 << 22)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        pts = sum(s["points_total"] for s in sums)
        m_d = 2 * ibmc.ibmc_ball_digits(r2)
        enumerated = len(P) * (35 * m_d + 595 * m_d * m_d)
        out[f"gamma_{gamma}"] = dict(radius_sq=r2, points_in_ball=int(pts), digit_points_enumerated=int(enumerated),
                                     seconds=round(t, 6), points_per_s=pts / t,
                                     us_per_image=round(t / len(P) * 1e6, 2),
                                     counterexamples=int(sum(s["cex_total"] for s in sums)),
                                     unsafe_images=int(sum(1 for s in sums if s["cex_total"] > 0)))
    out["workload"] = "glyph35 net 35-16-5, 10 glyphs, images within gamma * 255 (L2), k = 1..2"
    return out


def table_leg(ctx, ibmc, inputs):
    """The paper's threat to validity (Sec. IV-D: its CUDA code took the
    sigmoid from a table): the float version of the glyph35 net over the ten
    glyphs, deltas -16..16, k <= 2, checked with the exponential sigmoid and
    with the table sigmoid; the table's false counterexamples (records of the
    table check that the exponential check neither records nor flags as a
    near tie) and missed ones, and the two checks' times."""
    g = inputs.workload_glyph35()
    m = ibmc.Mlp(ctx, inputs.fnet_from_qnet(g.net))
    P = [(m, x, g.deltas, 1, 2) for x in g.images]
    out = {}
    recs = {}
    for name, tab in (("exp", False), ("table", True)):
        kw = dict(cex_capacity=1 << 22, near_tie_capacity=1 << 20, table_sigmoid=tab)
        ibmc.ibmc_check_batch(ctx, P, **kw)
        t0 = time.perf_counter()
        sums, cex, ties, _ = ibmc.ibmc_check_batch(ctx, P, **kw)
        t = time.perf_counter() - t0
        recs[name] = (set(zip(cex["prop"].tolist(), cex["k"].tolist(), cex["rank"].tolist())),
                      set(zip(ties["prop"].tolist(), ties["k"].tolist(), ties["rank"].tolist())))
        out[name] = dict(seconds=round(t, 6), points_per_s=sum(s["points_total"] for s in sums) / t,
                         counterexamples=len(recs[name][0]), near_ties=len(recs[name][1]))
    (e_rec, e_tie), (t_rec, t_tie) = recs["exp"], recs["table"]
    out["table_false_counterexamples"] = len(t_rec - e_rec - e_tie)
    out["table_missed_counterexamples"] = len(e_rec - t_rec - e_tie)
    out["workload"] = "glyph35 net as float sigmoid (W/64, b/16384), 10 glyphs, deltas -16..16, k = 1..2"
    # a property where the table does change verdicts: a seeded 35-16-5
    # float net (seed 25) on one glyph, the same domain
    g2 = inputs.rng(25)
    net2 = inputs.fnet_from_qnet(inputs.random_qnet(g2, [35, 16, 5], shift=7))
    x2 = inputs.glyph_images(g2, 1, 7, 5)[0]
    m2 = ibmc.Mlp(ctx, net2)
    sets = {}
    for name, tab in (("exp", False), ("table", True)):
        _, cx, tx = ibmc.ibmc_check_property(ctx, m2, x2, g.deltas, 1, 2, cex_capacity=1 << 22,
                                             near_tie_capacity=1 << 20, table_sigmoid=tab)
        sets[name] = (set(zip(cx["k"].tolist(), cx["rank"].tolist())), set(zip(tx["k"].tolist(), tx["rank"].tolist())))
    (e2, et2), (t2, _) = sets["exp"], sets["table"]
    out["seeded_property"] = dict(workload="35-16-5 float net (seed 25), one glyph, deltas -16..16, k = 1..2",
                                  exp_counterexamples=len(e2), table_counterexamples=len(t2),
                                  table_false_counterexamples=len(t2 - e2 - et2),
                                  table_missed_counterexamples=len(e2 - t2 - et2))
    return out


def train_flops(dims, samples):
    """Forward, weight-gradient and delta products of one pass (2 flops per
    multiply-add; no delta into the input layer)."""
    macs = sum(dims[l] * dims[l - 1] for l in range(1, len(dims)))
    return samples * 2 * (2 * macs + (macs - dims[1] * dims[0]))


def retrain_leg(ctx, ibmc, inputs):
    """Counterexample-augmented retraining (Sec. VI): a 35-16-10 float net
    trained on 400 labelled glyphs (10 classes a few pixels apart), checked
    on 12 of them (pixels flipped to 0 / 255, k = 1..2), retrained on the
    training set plus every counterexample with its clean label, checked
    again; and the training rate on 20,000 labelled glyphs."""
    g = inputs.rng(13)
    _, X, Y = inputs.labelled_glyphs(g, 10, 400, p_flip=0.03, proto_flip=0.15)
    net = inputs.random_fnet(g, [35, 16, 10])
    D = np.array([-255, 255], np.int16)
    t0 = time.perf_counter()
    m0, l0 = ibmc.ibmc_fit_mlp(ctx, ibmc.Mlp(ctx, net), X, Y, epochs=40, batch=32, lr=1e-2, seed=1)
    t_fit = time.perf_counter() - t0

    def check(mm):
        t = time.perf_counter()
        out = [ibmc.ibmc_check_property(ctx, mm, X[i], D, 1, 2)[1] for i in range(12)]
        return out, time.perf_counter() - t

    def augment(recs):
        ax, ay = [], []
        for i, cex in enumerate(recs):
            for k, r in zip(cex["k"], cex["rank"]):
                pix, dig = ibmc.ibmc_decode_point(35, 2, int(k), int(r))
                xp = X[i].astype(np.int64).copy()
                for p_, d_ in zip(pix, dig):
                    xp[p_] = min(255, max(0, xp[p_] + int(D[d_])))
                ax.append(xp.astype(np.uint8))
                ay.append(Y[i])
        return ax, ay

    before, t_chk = check(m0)
    aug_x, aug_y = augment(before)
    X2 = np.concatenate([X, np.stack(aug_x)]) if aug_x else X
    Y2 = np.concatenate([Y, np.array(aug_y, np.int32)])
    t0 = time.perf_counter()
    m1, l1 = ibmc.ibmc_fit_mlp(ctx, m0, X2, Y2, epochs=20, batch=32, lr=5e-3, seed=2)
    t_refit = time.perf_counter() - t0
    after, _ = check(m1)
    # a second pass of the loop on the counterexamples that remain
    ax2, ay2 = augment(after)
    if ax2:
        X3 = np.concatenate([X2, np.stack(ax2)])
        Y3 = np.concatenate([Y2, np.array(ay2, np.int32)])
        m2, _ = ibmc.ibmc_fit_mlp(ctx, m1, X3, Y3, epochs=20, batch=32, lr=5e-3, seed=3)
        second, _ = check(m2)
    else:
        second = after
    # training rate
    _, Xb, Yb = inputs.labelled_glyphs(g, 10, 20000, p_flip=0.03, proto_flip=0.15)
    rates = {}
    for dims in ([35, 16, 10], [35, 256, 128, 10]):
        mb = ibmc.Mlp(ctx, inputs.random_fnet(g, dims))
        ibmc.ibmc_fit_mlp(ctx, mb, Xb[:256], Yb[:256], epochs=1, batch=256, lr=1e-3)
        t0 = time.perf_counter()
        ibmc.ibmc_fit_mlp(ctx, mb, Xb, Yb, epochs=5, batch=256, lr=1e-3, seed=3)
        t = time.perf_counter() - t0
        tf = train_flops(dims, 5 * len(Yb)) / t / 1e12
        rates["-".join(map(str, dims))] = dict(samples_per_s=round(5 * len(Yb) / t), seconds=round(t, 4),
                                               tflops=round(tf, 4),
                                               frac_fp32_peak=round(tf / MI355X_FP32_PEAK_TFLOPS, 5))
    return dict(workload="35-16-10 float net, 400 labelled glyphs (10 classes), 12 properties, pixels to 0/255, "
                         "k = 1..2", counterexamples_before=int(sum(len(c) for c in before)),
                counterexamples_after=int(sum(len(c) for c in after)), augmented_samples=len(aug_x),
                counterexamples_after_second_pass=int(sum(len(c) for c in second)),
                loss_first_last=[round(float(l0[0]), 4), round(float(l0[-1]), 4)],
                fit_seconds=round(t_fit, 4), refit_seconds=round(t_refit, 4), check_seconds=round(t_chk, 4),
                training_rate_batch256=rates)


def replay_all(ibmc, ctx, net, w, cex):
    """Replays every counterexample record of the step (its point rebuilt from
    (k, rank) and the delta set, a full forward pass on the device) and counts
    the records whose replayed label equals the recorded one."""
    t0 = time.perf_counter()
    ok = 0
    order = np.argsort(cex["prop"], kind="stable")
    recs = cex[order]
    bounds = np.searchsorted(recs["prop"], np.arange(len(w.images) + 1))
    for i in range(len(w.images)):
        sel = recs[bounds[i]:bounds[i + 1]]
        if len(sel):
            ok += int(np.count_nonzero(ibmc.ibmc_replay(ctx, net, w.images[i], w.deltas, sel) == sel["new_label"]))
    return dict(records=int(len(cex)), replayed_ok=ok, seconds=round(time.perf_counter() - t0, 3))


def per_image(ibmc, ctx, net, w, sums):
    pots, labels = ibmc.ibmc_forward(ctx, net, w.images)
    z = np.sort(pots[:, -w.net.dims[-1]:].astype(np.int64), axis=1)
    return dict(counterexamples=[int(s["cex_total"]) for s in sums],
                clean_margin=[int(v) for v in (z[:, -1] - z[:, -2])])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--images", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", default=None)
    ap.add_argument("--no-extras", action="store_true", help="skip the proposer, coverage and batch legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the enumeration runs on a single device; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1907_12933_amd import ibmc, inputs

    w = inputs.workload_blob784(count=args.images)
    ctx = ibmc.Context(0, torch.cuda.current_stream())
    # the tuning table of this GPU (kernel choice per network shape), when shipped
    tuned = 0
    if os.path.exists(TUNE_TABLE):
        tuned = ibmc.ibmc_tune_load(ctx, TUNE_TABLE)
    net = ibmc.Mlp(ctx, w.net)
    if args.variant:
        ibmc.ibmc_set_variant(ctx, net, args.variant)
    imgs = torch.from_numpy(w.images).cuda()
    props = [(net, imgs[i], w.deltas, 1, 2) for i in range(args.images)]
    cap = 1 << 25
    # images and counterexample records both stay in HBM
    buf = torch.empty(cap * ibmc.CEX_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

    def step():
        return ibmc.ibmc_check_batch_dev(ctx, props, cex_capacity=cap, cex_buf=buf, records_on_device=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # objects alive now (torch's among them) leave the cyclic collector's
    # scans: a full collection over them stalls the host for tens of ms
    gc.collect()
    gc.freeze()
    ksec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sums, cex, _, rc = step()
        ks, nl = ibmc.ibmc_last_kernel_time(ctx)
        ksec.append(ks)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cex = np.frombuffer(cex.cpu().numpy().tobytes(), dtype=ibmc.CEX_DTYPE)
    points = sum(s["points_total"] for s in sums)
    value = points * args.steps / dt
    n_cex = sum(s["cex_total"] for s in sums)
    unsafe = sum(1 for s in sums if s["cex_total"] > 0)

    # roofline of the enumeration kernel: algorithmic int8 MACs per point are
    # the later layers' dense products (the first layer is the rank-k update);
    # its duration is the average of HIP events around the enumeration launch
    # alone, on the library's stream
    macs_per_point = dense_macs(w.net.dims)
    k_avg = float(np.mean(ksec))
    achieved_tops = 2.0 * macs_per_point * points / k_avg / 1e12
    prof = profile_record() if args.images == 64 else None
    roof = dict(bound="mfma", achieved=round(achieved_tops, 2), peak=MI355X_INT8_PEAK_TOPS, unit="TOP/s",
                frac=round(achieved_tops / MI355X_INT8_PEAK_TOPS, 4),
                traffic=prof["hbm_bytes_per_launch"] if prof else None,
                kernel="enum_q8", kernel_ms=round(k_avg * 1e3, 3),
                ops_per_point=2 * macs_per_point, points_per_launch=points)
    if prof:
        # the same figures from the committed rocprofv3 summaries of this
        # workload, and the ceiling at the shader clock measured there
        clk = prof["shader_clock_ghz"]
        roof.update(profile_kernel_ms=prof["kernel_trace_avg_ms"],
                    profile_frac=round(2.0 * macs_per_point * points / (prof["kernel_trace_avg_ms"] * 1e-3) / 1e12
                                       / MI355X_INT8_PEAK_TOPS, 4),
                    measured_clock_ghz=clk, peak_at_measured_clock=round(MI355X_INT8_PEAK_TOPS * clk /
                                                                         MI355X_SPEC_CLOCK_GHZ, 1),
                    frac_at_measured_clock=round(achieved_tops / (MI355X_INT8_PEAK_TOPS * clk /
                                                                  MI355X_SPEC_CLOCK_GHZ), 4),
                    mfma_busy=prof.get("mfma_busy"))
    out = {
        "metric": "perturbation points verified/sec + time-to-first-counterexample, plain vs learned",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": f"blob784: int8 MLP 784-256-256-10 (shift 7), {args.images} seeded 28x28 blob "
                               f"images, k=1..2 pixels, deltas +-8/+-16/+-32, all counterexamples returned",
                   "points_per_step": points, "images": args.images},
        "roofline": roof,
        "kernel": ibmc.ibmc_chosen_variant(ctx, net), "tuning_table_entries": tuned,
        "counterexamples_per_step": n_cex, "unsafe_images": unsafe,
        # per image: counterexamples and the clean top-2 logit margin
        "per_image": per_image(ibmc, ctx, net, w, sums),
        # every record of the last timed step replayed (after the timed region)
        "replay": replay_all(ibmc, ctx, net, w, cex),
    }
    if not args.no_extras:
        log("[bench] glyph leg")
        out["glyph35"] = glyph_leg(ctx, ibmc, inputs)
        log("[bench] coverage-guided test generation leg")
        out["coverage_search"] = covsearch_leg(ctx, ibmc, inputs)
        log("[bench] L2-ball leg")
        out["ball"] = ball_leg(ctx, ibmc, inputs)
        log("[bench] table sigmoid leg")
        out["table_sigmoid"] = table_leg(ctx, ibmc, inputs)
        log("[bench] proposer leg")
        out["ttfc"] = proposer_leg(ctx, ibmc, inputs, w, net, cex, args)
        log("[bench] coverage leg")
        out["coverage"] = coverage_leg(ctx, ibmc, inputs, torch)
        log("[bench] batch leg")
        out["batch"] = batch_leg(ctx, ibmc, inputs)
        log("[bench] retraining leg")
        out["retrain"] = retrain_leg(ctx, ibmc, inputs)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
