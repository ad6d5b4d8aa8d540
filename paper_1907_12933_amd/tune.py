"""Tune the enumeration kernel of every integer network the benchmark runs
(the 64-image blob784 step, the 35-16-5 glyph set and the eight networks of
the batched check) on this GPU, on the benchmark's own properties of that
network, and save the table next to the library (tune_gfx950.json), where
the benchmark loads it from.

Candidates are the kernels ibmc_autotune lists for the shape; each is timed
(device time of the whole batched check, best of three) on the properties
the benchmark gives that network, since the choice depends on the workload's
scale and delta sets as much as on the shape: on a few 10^6 points the
set-up of the persistent matrix-core grid dominates and the lane kernel
looks faster than it is on the 10^8-10^9 points of the benchmark.

    python -m paper_1907_12933_amd.tune [--out PATH]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT = os.path.join(HERE, "tune_gfx950.json")


def workloads():
    """(network, property list as (image, deltas, k_min, k_max)) per network."""
    from . import inputs as I
    w = I.workload_blob784()
    g = I.workload_glyph35()
    out = [(w.net, [(x, w.deltas, 1, 2) for x in w.images]), (g.net, [(x, g.deltas, 1, 2) for x in g.images])]
    nets, props = I.batch_workload(seed=3)
    for i, n in enumerate(nets):
        out.append((n, [(p.image, p.deltas, 1, p.k) for p in props if p.net_index == i]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT)
    args = ap.parse_args()
    import torch  # noqa: F401  (the HIP runtime torch uses)
    from . import ibmc
    ctx = ibmc.Context(0)
    table = {}
    for net, plist in workloads():
        m = ibmc.Mlp(ctx, net)
        rep = json.loads(ibmc.ibmc_autotune(ctx, m, k=1, n_deltas=2))   # the candidate list of the shape
        shape = rep["shape"]
        if shape in table:
            continue
        P = [(m, x, D, k0, k1) for x, D, k0, k1 in plist]
        times = {}
        for v in rep["variants"]:
            ibmc.ibmc_set_variant(ctx, m, v["name"])
            ibmc.ibmc_check_batch(ctx, P, cex_capacity=1 << 25)
            best = min(ibmc.ibmc_check_batch(ctx, P, cex_capacity=1 << 25)[0][0]["seconds"] for _ in range(3))
            times[v["name"]] = round(best * 1e3, 3)
        ibmc.ibmc_set_variant(ctx, m, None)
        table[shape] = min(times, key=times.get)
        print(shape, "->", table[shape], "ms:", times, flush=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=2, sort_keys=True)
        f.write("\n")
    print("saved", args.out, file=sys.stderr)


if __name__ == "__main__":
    main()
