"""Write full-size expected results computed by the CPU oracle only.

blob784_expected.json: for the images of the 784-256-256-10 blob workload
(k = 1, 2, deltas +-8/+-16/+-32; all 64 by default), the oracle's clean label,
per-level counterexample and exact-tie counts, and a SHA-256 of the sorted
(k, rank, new label) records.  Images are checked by the oracle's block-matrix
form (oracle/dense.py); an image already stored by the C oracle is
recomputed that way and must give the same record digest.
coverage784_expected.json: SS/DS/SV/DV coverage of the 784-1024-1024-1024-10
net over its 4,096 seeded pairs (counts and a SHA-256 of the bit array).
batch_expected.json: per listed property of the batched workload (the
784-512-512-10 ones at k = 2), the same fields as for blob784.
coverage784_65536_expected.json: the same net's coverage over the
benchmark's 65,536-pair sweep.

Usage: python tests/golden/make_expected.py [n_images] [--coverage] [--batch] [--sweep]
"""
import hashlib
import json
import multiprocessing
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import dense  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1907_12933_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def rec_digest(k, rank, label):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(k, np.int32).tobytes())
    h.update(np.ascontiguousarray(rank, np.int64).tobytes())
    h.update(np.ascontiguousarray(label, np.int32).tobytes())
    return h.hexdigest()


def blob784(n_images):
    path = os.path.join(HERE, "blob784_expected.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    w = I.workload_blob784()
    data["workload"] = "blob784 (seed 2): 784-256-256-10 shift 7, deltas +-8/+-16/+-32, k=1..2"
    data["net_sha256"] = w.net.digest()
    imgs = data.setdefault("images", {})
    todo = [i for i in range(n_images) if not (imgs.get(str(i)) or {}).get("oracle") == "dense"]
    # a few images at a time, each process with a share of the BLAS threads
    procs = int(os.environ.get("GOLDEN_PROCS", "4"))
    with multiprocessing.get_context("spawn").Pool(procs) as pool:
        for i, rec in pool.imap_unordered(_blob784_one, todo):
            old = imgs.get(str(i))
            _store(data, imgs, i, rec, old, path)


def _blob784_one(i):
    w = I.workload_blob784()
    t = time.time()
    r = dense.q8_check(w.net, w.images[i], w.deltas, 1, 2)
    return i, dict(image_sha256=I.array_digest(w.images[i]), clean_label=r["clean_label"],
                   cex=[int(v) for v in r["cex"]], ties=[int(v) for v in r["ties"]],
                   cex_total=r["cex_total"],
                   records_sha256=rec_digest(r["cex_k"], r["cex_rank"], r["cex_label"]),
                   first_records=[[int(a), int(b), int(c)] for a, b, c in
                                  zip(r["cex_k"][:5], r["cex_rank"][:5], r["cex_label"][:5])],
                   oracle="dense", oracle_seconds=round(time.time() - t, 1))


def _store(data, imgs, i, rec, old, path):
    if old:  # stored by the C oracle: both forms of the oracle must agree
        for key in ("image_sha256", "clean_label", "cex", "ties", "cex_total", "records_sha256"):
            assert old[key] == rec[key], (i, key, old[key], rec[key])
        rec["c_oracle_seconds"] = old["oracle_seconds"]
    imgs[str(i)] = rec
    print(i, rec["cex"], rec["oracle_seconds"], "(agrees with the C oracle)" if old else "", flush=True)
    data["images"] = dict(sorted(imgs.items(), key=lambda kv: int(kv[0])))
    json.dump(data, open(path, "w"), indent=1)


def coverage784():
    net, x1, x2 = I.coverage_pairs_blob784()
    t = time.time()
    P1 = np.stack([O.q8_forward(net, x)[0] for x in x1])
    P2 = np.stack([O.q8_forward(net, x)[0] for x in x2])
    out = dict(workload="coverage784 (seed 5): 784-1024-1024-1024-10 shift 7, 4096 pairs",
               net_sha256=net.digest(), pairs_sha256=I.array_digest(x1, x2), criteria={})
    for c in ("SS", "DS", "SV", "DV"):
        r = O.coverage(net.dims[1:], P1, P2, c)
        out["criteria"][c] = dict(covered_pairs=r["covered_pairs"], total_pairs=r["total_pairs"],
                                  covered_neurons=r["covered_neurons"], total_neurons=r["total_neurons"],
                                  literal=r["literal"], bits_sha256=hashlib.sha256(r["bits"].tobytes()).hexdigest())
        print(c, out["criteria"][c], flush=True)
    out["oracle_seconds"] = round(time.time() - t, 1)
    json.dump(out, open(os.path.join(HERE, "coverage784_expected.json"), "w"), indent=1)


def coverage784_sweep(n_pairs=65536):
    """The benchmark's 65,536-pair sweep: potentials by the block-matrix form
    of the oracle, coverage by the C oracle's literal predicates."""
    net, x1, x2 = I.coverage_pairs_blob784(n_pairs=n_pairs)
    t = time.time()
    P1 = dense.q8_potentials(net, x1)
    P2 = dense.q8_potentials(net, x2)
    out = dict(workload=f"coverage784 (seed 5): 784-1024-1024-1024-10 shift 7, {n_pairs} pairs",
               net_sha256=net.digest(), pairs_sha256=I.array_digest(x1, x2), criteria={})
    for c in ("SS", "DS", "SV", "DV"):
        r = O.coverage(net.dims[1:], P1, P2, c)
        out["criteria"][c] = dict(covered_pairs=r["covered_pairs"], total_pairs=r["total_pairs"],
                                  covered_neurons=r["covered_neurons"], total_neurons=r["total_neurons"],
                                  literal=r["literal"], bits_sha256=hashlib.sha256(r["bits"].tobytes()).hexdigest())
        print(c, out["criteria"][c], round(time.time() - t, 1), flush=True)
    out["oracle_seconds"] = round(time.time() - t, 1)
    json.dump(out, open(os.path.join(HERE, f"coverage784_{n_pairs}_expected.json"), "w"), indent=1)


# 784-512-512-10 properties at k = 2 of the benchmark's batched workload
BATCH_PROPS = (225, 226, 245)


def batch784():
    nets, props = I.batch_workload(seed=3)
    out = dict(workload="batch (seed 3): the 784-512-512-10 properties at k = 2 listed by index", props={})
    for i in BATCH_PROPS:
        p = props[i]
        net = nets[p.net_index]
        t = time.time()
        r = dense.q8_check(net, p.image, p.deltas, 1, p.k)
        out["props"][str(i)] = dict(
            net_sha256=net.digest(), dims=list(net.dims), image_sha256=I.array_digest(p.image),
            deltas=[int(d) for d in p.deltas], k=int(p.k), clean_label=r["clean_label"],
            points=[int(v) for v in r["points"]], cex=[int(v) for v in r["cex"]], ties=[int(v) for v in r["ties"]],
            records_sha256=rec_digest(r["cex_k"], r["cex_rank"], r["cex_label"]), oracle="dense",
            oracle_seconds=round(time.time() - t, 1))
        print(i, out["props"][str(i)]["cex"], out["props"][str(i)]["oracle_seconds"], flush=True)
    json.dump(out, open(os.path.join(HERE, "batch_expected.json"), "w"), indent=1)


if __name__ == "__main__":
    if "--sweep" in sys.argv:
        coverage784_sweep()
    if "--batch" in sys.argv or not os.path.exists(os.path.join(HERE, "batch_expected.json")):
        batch784()
    n = int(sys.argv[1]) if len(sys.argv) > 1 and sys.argv[1].isdigit() else 64
    if "--coverage" in sys.argv or not os.path.exists(os.path.join(HERE, "coverage784_expected.json")):
        coverage784()
    blob784(n)
