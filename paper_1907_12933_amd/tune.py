"""Tune the enumeration kernel of every integer network shape the benchmark
runs (the 64-image blob784 step, the 35-16-5 glyph set and the eight
networks of the batched check) on this GPU, and save the table next to the
library (tune_gfx950.json), where the benchmark loads it from.

    python -m paper_1907_12933_amd.tune [--out PATH]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT = os.path.join(HERE, "tune_gfx950.json")


def shapes():
    from . import inputs as I
    g = I.rng(1)
    nets = [I.workload_blob784(count=1).net, I.workload_glyph35().net]
    nets += [I.random_qnet(g, dims, shift=7) for dims in I.BATCH_TOPOLOGIES]
    return nets


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT)
    args = ap.parse_args()
    import torch  # noqa: F401  (the HIP runtime torch uses)
    from . import ibmc
    ctx = ibmc.Context(0)
    report = {}
    for net in shapes():
        m = ibmc.Mlp(ctx, net)
        # level 2 with enough points to keep the GPU busy: 33 deltas for the
        # small inputs, 6 for the 784-pixel ones
        rep = json.loads(ibmc.ibmc_autotune(ctx, m, k=2, n_deltas=33 if net.dims[0] <= 200 else 6))
        report[rep["shape"]] = {v["name"]: round(v["points_per_s"] / 1e9, 3) for v in rep["variants"]}
        print(rep["shape"], "->", rep["best"], report[rep["shape"]], flush=True)
    ibmc.ibmc_tune_save(ctx, args.out)
    print("saved", args.out, file=sys.stderr)


if __name__ == "__main__":
    main()
