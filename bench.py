"""Throughput of the exhaustive check on one MI355X.

Workload (one step): the 784-256-256-10 int8 network on 64 synthetic 28x28
blob images, every point with k = 1 and k = 2 changed pixels and deltas in
{+-8, +-16, +-32} (11,054,400 points per image, 707,481,600 per step), all
counterexamples returned to the host.  Images are resident in device memory
before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

MI355X_INT8_PEAK_TOPS = 5000.0     # dense int8 MFMA, TOP/s
MI355X_HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, target_seconds=15.0):
    """The oracle (plain full forward per point) on a seeded sample of the
    same workload's points: image 0, levels 1 and 2 in proportion."""
    from oracle import oracle as O
    n, m = w.net.dims[0], len(w.deltas)
    n1, n2 = O.points(n, m, 1), O.points(n, m, 2)
    g = np.random.Generator(np.random.PCG64(1234))
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    size = 20000
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
    return dict(value=total_pts / total_t, unit="points/s", cores=threads, kind="oracle",
                sample=f"{total_pts} seeded random points (k=1 and k=2 in proportion) of image 0, "
                       f"full int64 forward per point, {total_t:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--images", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1907_12933_amd import ibmc, inputs

    w = inputs.workload_blob784(count=args.images)
    ctx = ibmc.Context(0, torch.cuda.current_stream())
    net = ibmc.Mlp(ctx, w.net)
    if args.variant:
        ibmc.ibmc_set_variant(ctx, net, args.variant)
    imgs = torch.from_numpy(w.images).cuda()
    props = [(net, imgs[i], w.deltas, 1, 2) for i in range(args.images)]
    cap = 1 << 22

    def step():
        return ibmc.ibmc_check_batch_dev(ctx, props, cex_capacity=cap)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ksec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sums, cex, _, rc = step()
        ks, nl = ibmc.ibmc_last_kernel_time(ctx)
        ksec.append(ks)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    points = sum(s["points_total"] for s in sums)
    value = points * args.steps / dt
    n_cex = sum(s["cex_total"] for s in sums)
    unsafe = sum(1 for s in sums if s["cex_total"] > 0)

    # roofline of the enumeration kernel: algorithmic int8 MACs per point are
    # the later layers' dense products (the first layer is the rank-k update)
    d = w.net.dims
    macs_per_point = sum(d[l] * d[l + 1] for l in range(1, len(d) - 1))
    k_avg = float(np.mean(ksec))
    achieved_tops = 2.0 * macs_per_point * points / k_avg / 1e12
    roof = dict(bound="mfma", achieved=round(achieved_tops, 2), peak=MI355X_INT8_PEAK_TOPS, unit="TOP/s",
                frac=round(achieved_tops / MI355X_INT8_PEAK_TOPS, 4), traffic=None,
                kernel="enum_q8", kernel_ms=round(k_avg * 1e3, 3))
    out = {
        "metric": "perturbation points verified/sec + time-to-first-counterexample, plain vs learned",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": f"blob784: int8 MLP 784-256-256-10 (shift 7), {args.images} seeded 28x28 blob "
                               f"images, k=1..2 pixels, deltas +-8/+-16/+-32, all counterexamples returned",
                   "points_per_step": points, "images": args.images},
        "roofline": roof,
        "counterexamples_per_step": n_cex, "unsafe_images": unsafe,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
