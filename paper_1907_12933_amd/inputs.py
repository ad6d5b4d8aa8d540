"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and shapes them into networks, images,
delta sets and input pairs.  It holds none of the checking arithmetic (no
forward pass, no enumeration, no coverage predicate), so both the CPU oracle
and the HIP path can consume its output without sharing any of the method.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and draws integers
inclusively.  The workloads stand in for the paper's benchmark (5x5 vowel
glyphs classified by a small sigmoid MLP, Sec. IV-A): the glyphs and trained
weights are not published with the paper, so only their shapes are kept.

Network layout (plain numpy, row-major):
  ``dims``   list of L+1 widths: n_pixels, h1, ..., classes
  ``W[l]``   int8 [dims[l+1]][dims[l]]  (layer l+1 of the paper's Eq. (1))
  ``b[l]``   int32 [dims[l+1]]
  ``shift``  int32 per hidden layer (requantisation right shift)
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class QNet:
    dims: list
    W: list            # int8 arrays [dims[l+1], dims[l]]
    b: list            # int32 arrays [dims[l+1]]
    shift: list        # int per hidden layer

    @property
    def n_layers(self) -> int:
        return len(self.dims) - 1

    def dense_macs(self) -> int:
        """Multiply-accumulates of one full forward pass."""
        return sum(self.dims[i] * self.dims[i + 1] for i in range(self.n_layers))

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.asarray(self.dims, np.int64).tobytes())
        for w, b in zip(self.W, self.b):
            h.update(np.ascontiguousarray(w).tobytes())
            h.update(np.ascontiguousarray(b).tobytes())
        h.update(np.asarray(self.shift, np.int64).tobytes())
        return h.hexdigest()


@dataclasses.dataclass
class FNet:
    """Float32 network for the sigmoid variant (Sec. II-A, Eq. (2))."""
    dims: list
    W: list            # float32 [dims[l+1], dims[l]]
    b: list            # float32 [dims[l+1]]

    @property
    def n_layers(self) -> int:
        return len(self.dims) - 1


def random_qnet(g: np.random.Generator, dims, shift=7, wmax=64, bmax=512) -> QNet:
    dims = [int(d) for d in dims]
    W, b = [], []
    for l in range(len(dims) - 1):
        W.append(g.integers(-wmax, wmax, size=(dims[l + 1], dims[l]), endpoint=True).astype(np.int8))
        b.append(g.integers(-bmax, bmax, size=(dims[l + 1],), endpoint=True).astype(np.int32))
    if isinstance(shift, int):
        shift = [shift] * (len(dims) - 2)
    return QNet(dims, W, b, [int(s) for s in shift])


def fnet_from_qnet(q: QNet) -> FNet:
    """W/64 and b/16384 are exact in float32 for int8 / |b| < 2^24 integers."""
    return FNet(list(q.dims),
                [(w.astype(np.float32) / np.float32(64.0)).astype(np.float32) for w in q.W],
                [(b.astype(np.float32) / np.float32(16384.0)).astype(np.float32) for b in q.b])


def glyph_images(g: np.random.Generator, count: int, rows: int, cols: int, p_on=0.4) -> np.ndarray:
    """Binary glyph-like images: each pixel is 255 with probability p_on, else 0."""
    on = g.random((count, rows * cols)) < p_on
    return np.where(on, 255, 0).astype(np.uint8)


def labelled_glyphs(g: np.random.Generator, classes: int, count: int, rows: int = 7, cols: int = 5,
                    p_on=0.4, p_flip=0.05, proto_flip=None):
    """A labelled glyph set: `classes` random binary prototypes (as
    glyph_images; with proto_flip, one such base glyph with each pixel
    flipped with probability proto_flip per class, so that classes lie a
    few pixels apart); each sample copies a uniformly drawn prototype, flips
    each pixel with probability p_flip and takes the prototype's index as
    label.  Returns (prototypes [classes][rows*cols], images
    [count][rows*cols], labels int32 [count])."""
    if proto_flip is None:
        proto = glyph_images(g, classes, rows, cols, p_on)
    else:
        base = glyph_images(g, 1, rows, cols, p_on)[0]
        pf = g.random((classes, rows * cols)) < proto_flip
        proto = np.where(pf, 255 - base[None, :], base[None, :]).astype(np.uint8)
    labels = g.integers(0, classes - 1, size=count, endpoint=True).astype(np.int32)
    flip = g.random((count, rows * cols)) < p_flip
    imgs = np.where(flip, 255 - proto[labels], proto[labels]).astype(np.uint8)
    return proto, imgs, labels


def random_fnet(g: np.random.Generator, dims, scale=1.0) -> FNet:
    """Float32 network with weights normal(0, scale / sqrt(fan_in)) and zero biases."""
    W = [(g.standard_normal((dims[l + 1], dims[l])) * (scale / np.sqrt(dims[l]))).astype(np.float32)
         for l in range(len(dims) - 1)]
    b = [np.zeros(dims[l + 1], np.float32) for l in range(len(dims) - 1)]
    return FNet(list(dims), W, b)


def blob_images(g: np.random.Generator, count: int, side: int = 28, noise_std=20.0) -> np.ndarray:
    """28x28-shaped images: 1-3 Gaussian blobs plus uniform noise of the given std.

    Centres uniform in [4, side-5]^2, sigma uniform in [1.5, 4] pixels, amplitude
    uniform in [128, 255].  The noise is uniform on [-a, a] with a = std*sqrt(3);
    the sum is rounded to nearest and clamped to [0, 255].
    """
    yy, xx = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                         indexing="ij")
    out = np.empty((count, side * side), np.uint8)
    a = noise_std * math.sqrt(3.0)
    for i in range(count):
        img = np.zeros((side, side), np.float64)
        nb = int(g.integers(1, 3, endpoint=True))
        for _ in range(nb):
            cy, cx = g.uniform(4.0, side - 5.0, size=2)
            sig = g.uniform(1.5, 4.0)
            amp = g.uniform(128.0, 255.0)
            img += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sig * sig))
        img += g.uniform(-a, a, size=img.shape)
        out[i] = np.clip(np.rint(img), 0, 255).astype(np.uint8).reshape(-1)
    return out


def perturbed_partner(g: np.random.Generator, x1: np.ndarray, max_pixels: int, max_shift: int) -> np.ndarray:
    """x1 with m ~ U{1..max_pixels} distinct pixels shifted by U{-max_shift..max_shift}\\{0}, clamped."""
    x2 = x1.astype(np.int32).copy()
    m = int(g.integers(1, max_pixels, endpoint=True))
    pix = g.choice(x1.size, size=m, replace=False)
    for p in pix:
        d = 0
        while d == 0:
            d = int(g.integers(-max_shift, max_shift, endpoint=True))
        x2[p] = min(max(x2[p] + d, 0), 255)
    return x2.astype(np.uint8)


# --------------------------------------------------------------------------
# Workloads.  The sizes follow the benchmark configurations the build is
# measured on; see the module docstring for the relation to the paper.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class CheckWorkload:
    name: str
    net: QNet
    images: np.ndarray          # uint8 [count, n]
    deltas: np.ndarray          # int16 [m]
    k_max: int
    rows: int
    cols: int


def workload_glyph35(seed: int = 1) -> CheckWorkload:
    """35-16-5 ReLU net, ten 7x5 binary glyphs, deltas -16..16, k <= 2."""
    g = rng(seed)
    net = random_qnet(g, [35, 16, 5], shift=7)
    imgs = glyph_images(g, 10, 7, 5)
    deltas = np.arange(-16, 17, dtype=np.int16)
    return CheckWorkload("glyph35_35-16-5", net, imgs, deltas, 2, 7, 5)


def coverage_pairs_glyph35(seed: int = 1):
    """100 pairs for the 35-16-5 net: x1 = glyph[i mod 10], x2 = x1 with 1-8 shifted pixels."""
    w = workload_glyph35(seed)
    g = rng(seed * 1000 + 17)
    x1 = np.stack([w.images[i % 10] for i in range(100)])
    x2 = np.stack([perturbed_partner(g, x1[i], 8, 16) for i in range(100)])
    return w.net, x1, x2


def workload_blob784(seed: int = 2, count: int = 64) -> CheckWorkload:
    """784-256-256-10 net (shift 7), 64 blob images, deltas {+-8,+-16,+-32}, k <= 2."""
    g = rng(seed)
    net = random_qnet(g, [784, 256, 256, 10], shift=7)
    imgs = blob_images(g, count)
    deltas = np.array([-32, -16, -8, 8, 16, 32], dtype=np.int16)
    return CheckWorkload("blob784_784-256-256-10", net, imgs, deltas, 2, 28, 28)


def heldout_blob_images(seed: int = 40, count: int = 64) -> np.ndarray:
    return blob_images(rng(seed), count)


def coverage_pairs_blob784(seed: int = 5, n_pairs: int = 4096, dims=(784, 1024, 1024, 1024, 10)):
    """Wide 784-1024-1024-1024-10 net and blob pairs differing in 1-8 pixels by up to +-32."""
    g = rng(seed)
    net = random_qnet(g, list(dims), shift=7)
    x1 = blob_images(g, n_pairs)
    x2 = np.stack([perturbed_partner(g, x1[i], 8, 32) for i in range(n_pairs)])
    return net, x1, x2


DELTA_MENU = [
    [-8, 8],
    [-16, 16],
    [-16, -8, 8, 16],
    [-32, -16, -8, 8, 16, 32],
    list(range(-16, 17)),
]

BATCH_TOPOLOGIES = [
    [35, 16, 5], [35, 32, 16, 5], [64, 32, 10], [100, 64, 10],
    [196, 128, 64, 10], [784, 128, 10], [784, 256, 256, 10], [784, 512, 512, 10],
]

GRID = {35: (7, 5), 64: (8, 8), 100: (10, 10), 196: (14, 14), 784: (28, 28)}


def point_count(n: int, m: int, k: int) -> int:
    return math.comb(n, k) * m ** k


@dataclasses.dataclass
class Property:
    net_index: int
    image: np.ndarray
    deltas: np.ndarray
    k: int


def batch_workload(seed: int = 3, per_net: int = 32, mac_budget: float = 2e12):
    """Eight nets of uneven size, `per_net` properties each, k ~ U{1,2,3}.

    The delta set is drawn from DELTA_MENU.  A property whose plain-enumeration
    cost (points up to level k times the dense forward MACs) exceeds the budget
    first loses the pair of largest-|d| deltas while at least two deltas
    remain after the drop, then one level of k; a property still over budget
    at k = 1 stays as it is.
    """
    g = rng(seed)
    nets = [random_qnet(g, dims, shift=7) for dims in BATCH_TOPOLOGIES]
    props = []
    for ni, net in enumerate(nets):
        n = net.dims[0]
        r, c = GRID[n]
        for _ in range(per_net):
            k = int(g.integers(1, 3, endpoint=True))
            D = list(DELTA_MENU[int(g.integers(0, len(DELTA_MENU) - 1, endpoint=True))])
            if n <= 100:
                img = glyph_images(g, 1, r, c)[0]
            else:
                img = blob_images(g, 1, r)[0]
            macs = net.dense_macs()
            while sum(point_count(n, len(D), j) for j in range(1, k + 1)) * macs > mac_budget:
                big = max(abs(d) for d in D)
                rest = [d for d in D if abs(d) != big]
                if len(rest) >= 2:
                    D = rest
                elif k > 1:
                    k -= 1
                else:
                    break
            props.append(Property(ni, img, np.array(sorted(D), np.int16), k))
    return nets, props


def array_digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
