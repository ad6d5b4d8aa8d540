"""Plain-definition check of an integer network with whole-block matrix products.

TEST INFRASTRUCTURE ONLY: used by tests/ and by the script that writes the
stored expected results under tests/golden/.  The product library never
imports this module, and this module shares nothing with it.

What it computes is the same definition as ``oracle.q8_check`` (the C
oracle), written a second way so that the full-size workloads finish on a
workstation:

* the bounded domain of the incremental check (Sec. II-B: the bound grows
  level by level): at level k, every image that differs from the clean image
  x in exactly k pixels p1 < ... < pk, pixel pj set to
  clamp(x[pj] + D[ij], 0, 255); the point's rank is the lexicographic index
  of the pixel subset times |D|^k plus the delta indices read base |D| with
  i1 most significant;
* for every such image, the full forward pass of Eq. (1) (no incremental
  update): u_l = W_l a_{l-1} + b_l with a_0 = the pixels, hidden activations
  a = clamp(floor(u / 2^s), 0, 127), logits = the last layer's potentials;
* the safety property of Sec. III-C (Eq. (10) negated): a point is a
  counterexample when the lowest-index largest logit differs from the clean
  image's; an exact tie is a point whose largest logit is reached by more
  than one class.

The only step done by a library routine is the matrix product of a layer
over a block of points.  It runs in binary floating point, which is exact
here: every operand is an integer, and every partial sum of output j is
bounded by sum_i |W[j][i]| * max|a_i|.  When that bound is below 2^24
(float32) or 2^53 (float64), every partial sum and every rounding step is an
exact integer, whatever order the library adds in, so the product equals
the integer one.  The bound is checked per layer, and float32 is used only
where it holds.  The bias is added afterwards in int64.
"""
from __future__ import annotations

import itertools

import numpy as np


def _layer_dtype(W, max_in):
    """float32 when every output's partial sums stay below 2^24, float64 below 2^53."""
    bound = int(np.abs(W.astype(np.int64)).sum(axis=1).max()) * int(max_in)
    if bound < (1 << 24):
        return np.float32
    if bound < (1 << 53):
        return np.float64
    raise ValueError("layer partial sums exceed the exact range of float64")


class _Net:
    def __init__(self, net):
        self.W = [np.asarray(w, np.int64) for w in net.W]
        self.b = [np.asarray(b, np.int64) for b in net.b]
        self.shift = [int(s) for s in net.shift]
        self.L = len(self.W)
        self.dt = []
        self.WT = []
        for l, w in enumerate(self.W):
            dt = _layer_dtype(w, 255 if l == 0 else 127)
            self.dt.append(dt)
            self.WT.append(np.ascontiguousarray(w.T.astype(dt)))

    def potentials(self, X):
        """Potentials of every layer (int64 [B][sum of widths], layer by
        layer, Eq. (1)) of a block of images X (uint8 [B][n])."""
        a, out = X, []
        for l in range(self.L):
            u = np.rint(a.astype(self.dt[l]) @ self.WT[l]).astype(np.int64) + self.b[l]
            out.append(u)
            if l < self.L - 1:
                a = np.clip(np.floor_divide(u, 1 << self.shift[l]), 0, 127)
        return np.concatenate(out, axis=1)

    def logits(self, X):
        """Logits (int64 [B][classes]) of a block of images X (uint8 [B][n])."""
        a = X
        for l in range(self.L):
            u = np.rint(a.astype(self.dt[l]) @ self.WT[l]).astype(np.int64) + self.b[l]
            if l < self.L - 1:
                a = np.clip(np.floor_divide(u, 1 << self.shift[l]), 0, 127)
            else:
                return u


def _decide(z, clean):
    lab = np.argmax(z, axis=1)                       # lowest index of the largest logit
    top = z[np.arange(len(z)), lab]
    tie = (z == top[:, None]).sum(axis=1) > 1
    return lab, tie


def q8_check(net, x, deltas, k_min=1, k_max=2, k_step=1, block=8192):
    """Exhaustive integer check by the plain definition; the same result
    fields as the C oracle's q8_check (per-level points, counterexamples and
    exact ties, clean label, first unsafe level, records sorted by (k, rank))."""
    N = _Net(net)
    x = np.asarray(x, np.uint8)
    D = np.asarray(deltas, np.int64)
    n, m = x.size, D.size
    z0 = N.logits(x[None, :])
    clean = int(np.argmax(z0[0]))
    tie0 = int((z0[0] == z0[0].max()).sum() > 1)
    levels = list(range(k_min, k_max + 1, k_step))
    pts, cex, ties = [], [], []
    rk, rr, rl = [], [], []
    for k in levels:
        if k == 0:
            pts.append(1), cex.append(0), ties.append(tie0)
            continue
        mk = m ** k
        # delta-index tuples in rank order (i1 most significant)
        digits = np.array(list(itertools.product(range(m), repeat=k)), np.int64).reshape(mk, k)
        subsets = np.array(list(itertools.combinations(range(n), k)), np.int64).reshape(-1, k)
        per = max(1, block // mk)
        ncex = nties = 0
        for s0 in range(0, len(subsets), per):
            S = subsets[s0:s0 + per]
            B = len(S) * mk
            pix = np.repeat(S, mk, axis=0)                       # [B][k]
            dig = np.tile(digits, (len(S), 1))                   # [B][k]
            X = np.tile(x, (B, 1))
            rows = np.arange(B)[:, None]
            X[rows, pix] = np.clip(x[pix].astype(np.int64) + D[dig], 0, 255).astype(np.uint8)
            lab, tie = _decide(N.logits(X), clean)
            bad = np.nonzero(lab != clean)[0]
            ncex += bad.size
            nties += int(tie.sum())
            if bad.size:
                rank = (s0 + bad // mk) * mk + bad % mk
                rk.append(np.full(bad.size, k, np.int32))
                rr.append(rank.astype(np.int64))
                rl.append(lab[bad].astype(np.int32))
        pts.append(len(subsets) * mk)
        cex.append(ncex)
        ties.append(nties)
    first = next((k for k, c in zip(levels, cex) if c > 0), -1)
    cat = lambda v, t: np.concatenate(v).astype(t) if v else np.zeros(0, t)
    return dict(levels=levels, points=np.array(pts, np.int64), cex=np.array(cex, np.int64),
                ties=np.array(ties, np.int64), clean_label=clean, first_unsafe_k=first,
                cex_total=int(sum(cex)), cex_k=cat(rk, np.int32), cex_rank=cat(rr, np.int64),
                cex_label=cat(rl, np.int32))


def q8_potentials(net, X, block=4096):
    """Every layer's potentials (int64 [B][sum of widths]) of images X."""
    N = _Net(net)
    X = np.asarray(X, np.uint8).reshape(-1, net.dims[0])
    return np.concatenate([N.potentials(X[i:i + block]) for i in range(0, len(X), block)]) if len(X) else \
        np.zeros((0, sum(net.dims[1:])), np.int64)
