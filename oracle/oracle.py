"""ctypes front-end of the plain C oracle (ibmc_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke entry and the CPU-baseline
leg of the benchmark.  The product library never imports this module.
Every function here only marshals numpy arrays; the arithmetic is in C.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)
U64P = C.POINTER(C.c_uint64)
F64P = C.POINTER(C.c_double)
U8P = C.POINTER(C.c_uint8)
I8P = C.POINTER(C.c_int8)
I16P = C.POINTER(C.c_int16)

SS, DS, SV, DV = 0, 1, 2, 3
CRITERIA = {"SS": SS, "DS": DS, "SV": SV, "DV": DV, "VV": DV}


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.orc_q8_forward.argtypes = [C.c_int, I32P, I8P, I32P, I32P, U8P, I64P, I32P]
        L.orc_f64_forward.argtypes = [C.c_int, I32P, F64P, F64P, U8P, F64P, I32P, F64P]
        L.orc_points.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_points.restype = C.c_int64
        L.orc_decode.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, I32P, I32P]
        L.orc_q8_check.argtypes = [C.c_int, I32P, I8P, I32P, I32P, U8P, I16P, C.c_int,
                                   C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                   I64P, I64P, I64P, I32P, I32P, I32P, I64P, I32P, I64P, C.c_int]
        L.orc_ball_digits.argtypes = [C.c_int64]
        L.orc_q8_ball_check.argtypes = [C.c_int, I32P, I8P, I32P, I32P, U8P, C.c_int64,
                                        C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, I64P, I64P, I64P,
                                        I32P, I32P, I32P, I64P, I32P, I64P, C.c_int]
        L.orc_lut_sigmoid.argtypes = [C.c_double]
        L.orc_lut_sigmoid.restype = C.c_double
        L.orc_f64_check_ex.argtypes = [C.c_int, I32P, F64P, F64P, U8P, I16P, C.c_int,
                                       C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_double,
                                       C.c_int, C.c_int, C.c_double,
                                       I64P, I64P, I64P, I32P, I32P, I32P, I64P, I32P, I64P,
                                       C.c_int64, I32P, I64P, F64P, I64P, C.c_int]
        L.orc_q8_check_literal.argtypes = [C.c_int, I32P, I8P, I32P, I32P, U8P, I16P, C.c_int, C.c_int64,
                                           C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                           I64P, I64P, I64P, I32P, I32P, I32P, I64P, I32P, I64P, C.c_int]
        L.orc_f64_loss_grad.argtypes = [C.c_int, I32P, F64P, F64P, U8P, I32P, C.c_int64, F64P, F64P]
        L.orc_f64_check.argtypes = [C.c_int, I32P, F64P, F64P, U8P, I16P, C.c_int,
                                    C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_double,
                                    I64P, I64P, I64P, I32P, I32P, I32P, I64P, I32P, I64P,
                                    C.c_int64, I32P, I64P, F64P, I64P, C.c_int]
        L.orc_q8_eval_points.argtypes = [C.c_int, I32P, I8P, I32P, I32P, U8P, I16P, C.c_int,
                                         I32P, I64P, C.c_int64, I32P, I64P, C.c_int]
        L.orc_f64_eval_points.argtypes = [C.c_int, I32P, F64P, F64P, U8P, I16P, C.c_int,
                                          I32P, I64P, C.c_int64, I32P, F64P, F64P, C.c_int]
        L.orc_coverage.argtypes = [C.c_int, I32P, I64P, I64P, C.c_int64, C.c_int, C.c_int64,
                                   C.c_int32, C.c_int32, C.c_double, U64P, I64P, F64P, I32P]
        L.orc_euclid.argtypes = [F64P, F64P, C.c_int64]
        L.orc_euclid.restype = C.c_double
        L.orc_prop_loss_grad.argtypes = [C.c_int, C.c_int, C.c_int, F64P, F64P, C.c_double,
                                         F64P, F64P, F64P, C.c_double, F64P, F64P, F64P, F64P,
                                         F64P, F64P]
        L.orc_adam_step.argtypes = [C.c_int64, F64P, F64P, F64P, F64P, C.c_int, C.c_double,
                                    C.c_double, C.c_double, C.c_double]
        L.orc_adam_step.restype = None
        L.orc_prop_features.argtypes = [C.c_int, I32P, I8P, I32P, I32P, U8P, C.c_int, C.c_int, I16P, C.c_int, F64P]
        _LIB = L
    return _LIB


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


class OracleError(RuntimeError):
    pass


def _ck(rc):
    if rc < 0:
        raise OracleError(f"oracle call failed with code {rc}")
    return rc


def _flat_q8(net):
    dims = np.ascontiguousarray(net.dims, np.int32)
    W = np.concatenate([np.ascontiguousarray(w, np.int8).reshape(-1) for w in net.W])
    b = np.concatenate([np.ascontiguousarray(x, np.int32).reshape(-1) for x in net.b])
    sh = np.ascontiguousarray(list(net.shift) + [0], np.int32)
    return dims, W, b, sh


def _flat_f64(net):
    dims = np.ascontiguousarray(net.dims, np.int32)
    W = np.concatenate([np.asarray(w, np.float64).reshape(-1) for w in net.W])
    b = np.concatenate([np.asarray(x, np.float64).reshape(-1) for x in net.b])
    return dims, W, b


def q8_forward(net, x):
    """All potentials (layers 1..L concatenated, int64) and the label of image x."""
    dims, W, b, sh = _flat_q8(net)
    x = np.ascontiguousarray(x, np.uint8)
    pot = np.zeros(int(sum(net.dims[1:])), np.int64)
    lab = np.zeros(1, np.int32)
    _ck(lib().orc_q8_forward(len(dims) - 1, _p(dims, I32P), _p(W, I8P), _p(b, I32P), _p(sh, I32P),
                             _p(x, U8P), _p(pot, I64P), _p(lab, I32P)))
    return pot, int(lab[0])


def f64_forward(net, x):
    dims, W, b = _flat_f64(net)
    x = np.ascontiguousarray(x, np.uint8)
    pot = np.zeros(int(sum(net.dims[1:])), np.float64)
    lab = np.zeros(1, np.int32)
    mg = np.zeros(1, np.float64)
    _ck(lib().orc_f64_forward(len(dims) - 1, _p(dims, I32P), _p(W, F64P), _p(b, F64P), _p(x, U8P),
                              _p(pot, F64P), _p(lab, I32P), _p(mg, F64P)))
    return pot, int(lab[0]), float(mg[0])


def points(n, m, k):
    return int(lib().orc_points(n, m, k))


def decode(n, m, k, rank):
    pix = np.zeros(max(k, 1), np.int32)
    dig = np.zeros(max(k, 1), np.int32)
    _ck(lib().orc_decode(n, m, k, int(rank), _p(pix, I32P), _p(dig, I32P)))
    return pix[:k].copy(), dig[:k].copy()


def _levels(k_min, k_max, k_step):
    return len(range(k_min, k_max + 1, k_step))


def q8_check(net, x, deltas, k_min=1, k_max=2, k_step=1, stop_at_first=False, cap=1 << 22,
             nthreads=None):
    """Exhaustive integer check.  Returns a dict with per-level points / cex / exact ties,
    the clean label, the first unsafe k, and the sorted counterexample arrays."""
    dims, W, b, sh = _flat_q8(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    nl = _levels(k_min, k_max, k_step)
    pts = np.zeros(nl, np.int64); cx = np.zeros(nl, np.int64); ti = np.zeros(nl, np.int64)
    cl = np.zeros(1, np.int32); fu = np.zeros(1, np.int32)
    ok = np.zeros(cap, np.int32); orr = np.zeros(cap, np.int64); ol = np.zeros(cap, np.int32)
    nout = np.zeros(1, np.int64)
    lev = _ck(lib().orc_q8_check(len(dims) - 1, _p(dims, I32P), _p(W, I8P), _p(b, I32P), _p(sh, I32P),
                                 _p(x, U8P), _p(D, I16P), len(D), k_min, k_max, k_step,
                                 int(stop_at_first), cap, _p(pts, I64P), _p(cx, I64P), _p(ti, I64P),
                                 _p(cl, I32P), _p(fu, I32P), _p(ok, I32P), _p(orr, I64P), _p(ol, I32P),
                                 _p(nout, I64P), _threads(nthreads)))
    n = int(nout[0]); w = min(n, cap)
    return dict(levels=list(range(k_min, k_max + 1, k_step))[:lev], points=pts[:lev], cex=cx[:lev],
                ties=ti[:lev], clean_label=int(cl[0]), first_unsafe_k=int(fu[0]), cex_total=n,
                cex_k=ok[:w].copy(), cex_rank=orr[:w].copy(), cex_label=ol[:w].copy())


def ball_digits(r2):
    """Digits per pixel of the L2-ball encoding: m = 2 * ball_digits(r2)."""
    return int(lib().orc_ball_digits(int(r2)))


def q8_ball_check(net, x, r2, k_min=1, k_max=2, k_step=1, stop_at_first=False, cap=1 << 22, nthreads=None):
    """Exhaustive integer check over the images within squared L2 distance r2
    of x, level k = support size.  Same result layout as q8_check."""
    dims, W, b, sh = _flat_q8(net)
    x = np.ascontiguousarray(x, np.uint8)
    nl = _levels(k_min, k_max, k_step)
    pts = np.zeros(nl, np.int64); cx = np.zeros(nl, np.int64); ti = np.zeros(nl, np.int64)
    cl = np.zeros(1, np.int32); fu = np.zeros(1, np.int32)
    ok = np.zeros(cap, np.int32); orr = np.zeros(cap, np.int64); ol = np.zeros(cap, np.int32)
    nout = np.zeros(1, np.int64)
    lev = _ck(lib().orc_q8_ball_check(len(dims) - 1, _p(dims, I32P), _p(W, I8P), _p(b, I32P), _p(sh, I32P),
                                      _p(x, U8P), int(r2), k_min, k_max, k_step, int(stop_at_first), cap,
                                      _p(pts, I64P), _p(cx, I64P), _p(ti, I64P), _p(cl, I32P), _p(fu, I32P),
                                      _p(ok, I32P), _p(orr, I64P), _p(ol, I32P), _p(nout, I64P),
                                      _threads(nthreads)))
    n = int(nout[0]); w = min(n, cap)
    return dict(levels=list(range(k_min, k_max + 1, k_step))[:lev], points=pts[:lev], cex=cx[:lev],
                ties=ti[:lev], clean_label=int(cl[0]), first_unsafe_k=int(fu[0]), cex_total=n,
                cex_k=ok[:w].copy(), cex_rank=orr[:w].copy(), cex_label=ol[:w].copy(), m=2 * ball_digits(r2))


def f64_loss_grad(net, images, labels):
    """Mean softmax cross-entropy of the float network on labelled images and
    its gradient over theta (per layer W row-major, then b)."""
    dims, W, b = _flat_f64(net)
    images = np.ascontiguousarray(images, np.uint8).reshape(-1, net.dims[0])
    labels = np.ascontiguousarray(labels, np.int32)
    P = sum(net.dims[l] * net.dims[l - 1] + net.dims[l] for l in range(1, len(net.dims)))
    g = np.zeros(P, np.float64)
    loss = np.zeros(1, np.float64)
    _ck(lib().orc_f64_loss_grad(len(dims) - 1, _p(dims, I32P), _p(W, F64P), _p(b, F64P), _p(images, U8P),
                                _p(labels, I32P), len(labels), _p(g, F64P), _p(loss, F64P)))
    return float(loss[0]), g


def f64_fit(net, images, labels, order, batch, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Mini-batch Adam (Kingma and Ba, Algorithm 1) on the mean loss of each
    batch: epoch e visits images order[e] in consecutive batches of `batch`.
    Returns (W list, b list, mean loss of each epoch's batches before their
    steps), all in double."""
    dims = list(net.dims)
    W = [np.asarray(w, np.float64).copy() for w in net.W]
    b = [np.asarray(x, np.float64).copy() for x in net.b]
    theta = np.concatenate([np.concatenate([w.reshape(-1), x]) for w, x in zip(W, b)])
    images = np.ascontiguousarray(images, np.uint8).reshape(-1, dims[0])
    labels = np.asarray(labels, np.int32)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t = 0
    losses = []

    def unflat(th):
        Ws, bs, o = [], [], 0
        for l in range(1, len(dims)):
            nw = dims[l] * dims[l - 1]
            Ws.append(th[o:o + nw].reshape(dims[l], dims[l - 1]))
            o += nw
            bs.append(th[o:o + dims[l]])
            o += dims[l]
        return Ws, bs

    class _Net:
        pass
    for ord_e in np.asarray(order, np.int64):
        total = 0.0
        for b0 in range(0, len(ord_e), batch):
            idx = ord_e[b0:b0 + batch]
            cur = _Net()
            cur.dims = dims
            cur.W, cur.b = unflat(theta)
            loss, g = f64_loss_grad(cur, images[idx], labels[idx])
            total += loss * len(idx)
            t += 1
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            mhat = m / (1 - beta1 ** t)
            vhat = v / (1 - beta2 ** t)
            theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
        losses.append(total / len(ord_e))
    Ws, bs = unflat(theta)
    return [w.copy() for w in Ws], [x.copy() for x in bs], np.array(losses)


def lut_sigmoid(u):
    """The table sigmoid (knots -8 + i/16, FP32 values, linear between)."""
    return float(lib().orc_lut_sigmoid(float(u)))


def q8_check_literal(net, x, deltas, V, k_min=1, k_max=2, k_step=1, stop_at_first=False, cap=1 << 22,
                     nthreads=None):
    """Integer check of the threshold literal (z_D < V and max_{i != D} z_i > V)."""
    dims, W, b, sh = _flat_q8(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    nl = _levels(k_min, k_max, k_step)
    pts = np.zeros(nl, np.int64); cx = np.zeros(nl, np.int64); ti = np.zeros(nl, np.int64)
    cl = np.zeros(1, np.int32); fu = np.zeros(1, np.int32)
    ok = np.zeros(cap, np.int32); orr = np.zeros(cap, np.int64); ol = np.zeros(cap, np.int32)
    nout = np.zeros(1, np.int64)
    lev = _ck(lib().orc_q8_check_literal(len(dims) - 1, _p(dims, I32P), _p(W, I8P), _p(b, I32P), _p(sh, I32P),
                                         _p(x, U8P), _p(D, I16P), len(D), int(V), k_min, k_max, k_step,
                                         int(stop_at_first), cap, _p(pts, I64P), _p(cx, I64P), _p(ti, I64P),
                                         _p(cl, I32P), _p(fu, I32P), _p(ok, I32P), _p(orr, I64P), _p(ol, I32P),
                                         _p(nout, I64P), _threads(nthreads)))
    n = int(nout[0]); w = min(n, cap)
    return dict(levels=list(range(k_min, k_max + 1, k_step))[:lev], points=pts[:lev], cex=cx[:lev],
                ties=ti[:lev], clean_label=int(cl[0]), first_unsafe_k=int(fu[0]), cex_total=n,
                cex_k=ok[:w].copy(), cex_rank=orr[:w].copy(), cex_label=ol[:w].copy())


def f64_check(net, x, deltas, k_min=1, k_max=2, k_step=1, stop_at_first=False, cap=1 << 22,
              tie_rel=4e-5, tie_cap=1 << 22, nthreads=None, lut=False, literal_v=None):
    """Double-precision float check; lut: the table sigmoid; literal_v: check
    the threshold literal with this reference value instead of the label."""
    if lut or literal_v is not None:
        return _f64_check_ex(net, x, deltas, k_min, k_max, k_step, stop_at_first, cap, tie_rel, tie_cap,
                             nthreads, lut, literal_v)
    dims, W, b = _flat_f64(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    nl = _levels(k_min, k_max, k_step)
    pts = np.zeros(nl, np.int64); cx = np.zeros(nl, np.int64); ti = np.zeros(nl, np.int64)
    cl = np.zeros(1, np.int32); fu = np.zeros(1, np.int32)
    ok = np.zeros(cap, np.int32); orr = np.zeros(cap, np.int64); ol = np.zeros(cap, np.int32)
    tk = np.zeros(tie_cap, np.int32); tr = np.zeros(tie_cap, np.int64); tm = np.zeros(tie_cap, np.float64)
    nout = np.zeros(1, np.int64); ntie = np.zeros(1, np.int64)
    lev = _ck(lib().orc_f64_check(len(dims) - 1, _p(dims, I32P), _p(W, F64P), _p(b, F64P), _p(x, U8P),
                                  _p(D, I16P), len(D), k_min, k_max, k_step, int(stop_at_first), cap,
                                  float(tie_rel), _p(pts, I64P), _p(cx, I64P), _p(ti, I64P),
                                  _p(cl, I32P), _p(fu, I32P), _p(ok, I32P), _p(orr, I64P), _p(ol, I32P),
                                  _p(nout, I64P), tie_cap, _p(tk, I32P), _p(tr, I64P), _p(tm, F64P),
                                  _p(ntie, I64P), _threads(nthreads)))
    n = int(nout[0]); w = min(n, cap)
    nt = int(ntie[0]); wt = min(nt, tie_cap)
    return dict(levels=list(range(k_min, k_max + 1, k_step))[:lev], points=pts[:lev], cex=cx[:lev],
                ties=ti[:lev], clean_label=int(cl[0]), first_unsafe_k=int(fu[0]), cex_total=n,
                cex_k=ok[:w].copy(), cex_rank=orr[:w].copy(), cex_label=ol[:w].copy(),
                tie_total=nt, tie_k=tk[:wt].copy(), tie_rank=tr[:wt].copy(), tie_margin=tm[:wt].copy())


def _f64_check_ex(net, x, deltas, k_min, k_max, k_step, stop_at_first, cap, tie_rel, tie_cap, nthreads, lut,
                  literal_v):
    dims, W, b = _flat_f64(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    nl = _levels(k_min, k_max, k_step)
    pts = np.zeros(nl, np.int64); cx = np.zeros(nl, np.int64); ti = np.zeros(nl, np.int64)
    cl = np.zeros(1, np.int32); fu = np.zeros(1, np.int32)
    ok = np.zeros(cap, np.int32); orr = np.zeros(cap, np.int64); ol = np.zeros(cap, np.int32)
    tk = np.zeros(tie_cap, np.int32); tr = np.zeros(tie_cap, np.int64); tm = np.zeros(tie_cap, np.float64)
    nout = np.zeros(1, np.int64); ntie = np.zeros(1, np.int64)
    lev = _ck(lib().orc_f64_check_ex(len(dims) - 1, _p(dims, I32P), _p(W, F64P), _p(b, F64P), _p(x, U8P),
                                     _p(D, I16P), len(D), k_min, k_max, k_step, int(stop_at_first), cap,
                                     float(tie_rel), int(bool(lut)), int(literal_v is not None),
                                     float(literal_v or 0.0), _p(pts, I64P), _p(cx, I64P), _p(ti, I64P),
                                     _p(cl, I32P), _p(fu, I32P), _p(ok, I32P), _p(orr, I64P), _p(ol, I32P),
                                     _p(nout, I64P), tie_cap, _p(tk, I32P), _p(tr, I64P), _p(tm, F64P),
                                     _p(ntie, I64P), _threads(nthreads)))
    n = int(nout[0]); w = min(n, cap)
    nt = int(ntie[0]); wt = min(nt, tie_cap)
    return dict(levels=list(range(k_min, k_max + 1, k_step))[:lev], points=pts[:lev], cex=cx[:lev],
                ties=ti[:lev], clean_label=int(cl[0]), first_unsafe_k=int(fu[0]), cex_total=n,
                cex_k=ok[:w].copy(), cex_rank=orr[:w].copy(), cex_label=ol[:w].copy(),
                tie_total=nt, tie_k=tk[:wt].copy(), tie_rank=tr[:wt].copy(), tie_margin=tm[:wt].copy())


def q8_eval_points(net, x, deltas, ks, ranks, want_logits=False, nthreads=None):
    dims, W, b, sh = _flat_q8(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    ks = np.ascontiguousarray(ks, np.int32); ranks = np.ascontiguousarray(ranks, np.int64)
    n = len(ks)
    labels = np.zeros(n, np.int32)
    logits = np.zeros((n, net.dims[-1]), np.int64) if want_logits else None
    _ck(lib().orc_q8_eval_points(len(dims) - 1, _p(dims, I32P), _p(W, I8P), _p(b, I32P), _p(sh, I32P),
                                 _p(x, U8P), _p(D, I16P), len(D), _p(ks, I32P), _p(ranks, I64P), n,
                                 _p(labels, I32P), _p(logits, I64P), _threads(nthreads)))
    return (labels, logits) if want_logits else labels


def f64_eval_points(net, x, deltas, ks, ranks, nthreads=None):
    dims, W, b = _flat_f64(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    ks = np.ascontiguousarray(ks, np.int32); ranks = np.ascontiguousarray(ranks, np.int64)
    n = len(ks)
    labels = np.zeros(n, np.int32)
    logits = np.zeros((n, net.dims[-1]), np.float64)
    margins = np.zeros(n, np.float64)
    _ck(lib().orc_f64_eval_points(len(dims) - 1, _p(dims, I32P), _p(W, F64P), _p(b, F64P), _p(x, U8P),
                                  _p(D, I16P), len(D), _p(ks, I32P), _p(ranks, I64P), n,
                                  _p(labels, I32P), _p(logits, F64P), _p(margins, F64P),
                                  _threads(nthreads)))
    return labels, logits, margins


def coverage(widths, pot1, pot2, criterion, dist_sq_min=1, ratio_num=3, ratio_den=2, P=0.8):
    """Literal SS/DS/SV/DV coverage.  pot1/pot2: int64 [n_pairs, sum(widths)]."""
    widths = np.ascontiguousarray(widths, np.int32)
    pot1 = np.ascontiguousarray(pot1, np.int64).reshape(-1)
    pot2 = np.ascontiguousarray(pot2, np.int64).reshape(-1)
    U = int(widths.sum())
    npairs = pot1.size // U if U else 0
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    tp = sum(int(widths[i]) * int(widths[i + 1]) for i in range(len(widths) - 1))
    bits = np.zeros(max((tp + 63) // 64, 1), np.uint64)
    counts = np.zeros(4, np.int64); frac = np.zeros(1, np.float64); lit = np.zeros(1, np.int32)
    _ck(lib().orc_coverage(len(widths), _p(widths, I32P), _p(pot1, I64P), _p(pot2, I64P), npairs, crit,
                           int(dist_sq_min), int(ratio_num), int(ratio_den), float(P), _p(bits, U64P),
                           _p(counts, I64P), _p(frac, F64P), _p(lit, I32P)))
    return dict(covered_pairs=int(counts[0]), total_pairs=int(counts[1]), covered_neurons=int(counts[2]),
                total_neurons=int(counts[3]), fraction=float(frac[0]), literal=bool(lit[0]),
                bits=bits[:(tp + 63) // 64].copy())


def euclid(p, q):
    p = np.ascontiguousarray(p, np.float64); q = np.ascontiguousarray(q, np.float64)
    return float(lib().orc_euclid(_p(p, F64P), _p(q, F64P), p.size))


def prop_loss_grad(f, y, pw, W1, b1, w2, c):
    f = np.ascontiguousarray(f, np.float64); y = np.ascontiguousarray(y, np.float64)
    W1 = np.ascontiguousarray(W1, np.float64); b1 = np.ascontiguousarray(b1, np.float64)
    w2 = np.ascontiguousarray(w2, np.float64)
    B, F = f.shape
    H = W1.shape[0]
    loss = np.zeros(1); gW1 = np.zeros_like(W1); gb1 = np.zeros_like(b1); gw2 = np.zeros_like(w2)
    gc = np.zeros(1); s = np.zeros(B)
    _ck(lib().orc_prop_loss_grad(B, F, H, _p(f, F64P), _p(y, F64P), float(pw), _p(W1, F64P),
                                 _p(b1, F64P), _p(w2, F64P), float(c), _p(loss, F64P), _p(gW1, F64P),
                                 _p(gb1, F64P), _p(gw2, F64P), _p(gc, F64P), _p(s, F64P)))
    return dict(loss=float(loss[0]), W1=gW1, b1=gb1, w2=gw2, c=float(gc[0]), scores=s)


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays theta, m, v."""
    for a in (theta, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam_step(theta.size, _p(theta, F64P), _p(g, F64P), _p(m, F64P), _p(v, F64P), int(t),
                        float(lr), float(beta1), float(beta2), float(eps))


def prop_features(net, x, rows, cols, deltas):
    """Candidate features [n * |D|, 32] (double) of image x for the proposal network."""
    dims, W, b, sh = _flat_q8(net)
    x = np.ascontiguousarray(x, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    f = np.zeros((x.size * D.size, 32), np.float64)
    _ck(lib().orc_prop_features(len(dims) - 1, _p(dims, I32P), _p(W, I8P), _p(b, I32P), _p(sh, I32P), _p(x, U8P),
                                int(rows), int(cols), _p(D, I16P), D.size, _p(f, F64P)))
    return f
