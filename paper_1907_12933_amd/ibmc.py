"""ctypes binding of libibmc.so (the C ABI in include/ibmc.h), same names.

Argument marshalling only: every step of the check and of the coverage runs
in the library's HIP kernels.  PyTorch is used, where a caller wants it, for
device memory (the *_dev calls take torch tensors) and for the stream a
context runs on.  There is no CPU fallback: if the library is missing,
loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibmc.so")

IBMC_OK = 0
IBMC_W_TRUNCATED = 1
IBMC_W_PARTIAL = 2
IBMC_E_INVALID = -1
IBMC_E_RANGE = -2
IBMC_E_HIP = -3
IBMC_E_OOM = -4
IBMC_E_ABORTED = -5
IBMC_E_UNIMPL = -6
IBMC_MAX_LEVELS = 16
IBMC_ACT_RELU_Q8 = 0
IBMC_ACT_SIGMOID_F32 = 1
IBMC_COV_SS, IBMC_COV_DS, IBMC_COV_SV, IBMC_COV_DV = 0, 1, 2, 3
IBMC_COV_VV = IBMC_COV_DV
CRITERIA = {"SS": 0, "DS": 1, "SV": 2, "DV": 3, "VV": 3}
PROP_FEATURES = 32
PROP_HIDDEN = 128


class IbmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ibmc error {code}: {msg}")
        self.code = code


class ibmc_mlp_desc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.POINTER(C.c_int32)), ("act", C.c_int32),
                ("W", C.POINTER(C.c_void_p)), ("b", C.POINTER(C.c_void_p)), ("shift", C.POINTER(C.c_int32))]


class ibmc_check_opts(C.Structure):
    _fields_ = [("k_min", C.c_int32), ("k_max", C.c_int32), ("k_step", C.c_int32),
                ("stop_at_first", C.c_int32), ("cex_capacity", C.c_int64),
                ("near_tie_capacity", C.c_int64), ("near_tie_rel", C.c_float), ("records_on_device", C.c_int32),
                ("resume_cursor", C.c_int64), ("chunk_budget", C.c_int64), ("property", C.c_int32),
                ("sigmoid", C.c_int32), ("literal_v", C.c_double)]


class ibmc_cex(C.Structure):
    _fields_ = [("prop", C.c_int32), ("k", C.c_int32), ("rank", C.c_int64), ("new_label", C.c_int32),
                ("reserved", C.c_int32)]


CEX_DTYPE = np.dtype([("prop", np.int32), ("k", np.int32), ("rank", np.int64), ("new_label", np.int32),
                      ("reserved", np.int32)])
assert CEX_DTYPE.itemsize == C.sizeof(ibmc_cex)


class ibmc_check_summary(C.Structure):
    _fields_ = [("clean_label", C.c_int32), ("first_unsafe_k", C.c_int32), ("n_levels", C.c_int32),
                ("safe_up_to_k", C.c_int32), ("level_k", C.c_int32 * IBMC_MAX_LEVELS),
                ("points", C.c_int64 * IBMC_MAX_LEVELS), ("cex", C.c_int64 * IBMC_MAX_LEVELS),
                ("ties", C.c_int64 * IBMC_MAX_LEVELS), ("points_total", C.c_int64), ("cex_total", C.c_int64),
                ("near_ties_total", C.c_int64), ("seconds", C.c_double), ("ttfc_seconds", C.c_double),
                ("points_before_first", C.c_int64), ("next_cursor", C.c_int64)]


class ibmc_property(C.Structure):
    _fields_ = [("net", C.c_void_p), ("image", C.c_void_p), ("deltas", C.POINTER(C.c_int16)),
                ("n_deltas", C.c_int32), ("k_min", C.c_int32), ("k_max", C.c_int32), ("k_step", C.c_int32)]


class ibmc_ball_property(C.Structure):
    _fields_ = [("net", C.c_void_p), ("image", C.c_void_p), ("radius_sq", C.c_int64), ("k_min", C.c_int32),
                ("k_max", C.c_int32), ("k_step", C.c_int32), ("reserved", C.c_int32)]


class ibmc_cov_params(C.Structure):
    _fields_ = [("dist_sq_min", C.c_int64), ("ratio_num", C.c_int32), ("ratio_den", C.c_int32), ("P", C.c_double)]


class ibmc_cov_summary(C.Structure):
    _fields_ = [("covered_pairs", C.c_int64), ("total_pairs", C.c_int64), ("covered_neurons", C.c_int64),
                ("total_neurons", C.c_int64), ("fraction", C.c_double), ("literal", C.c_int32),
                ("reserved", C.c_int32), ("seconds", C.c_double)]


class ibmc_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("pos_weight", C.c_float), ("seed", C.c_uint64)]


class ibmc_fit_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64), ("order", C.POINTER(C.c_int64))]


VP = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
P_I32 = C.POINTER(C.c_int32)
P_I64 = C.POINTER(C.c_int64)
P_I16 = C.POINTER(C.c_int16)
P_U8 = C.POINTER(C.c_uint8)
P_U64 = C.POINTER(C.c_uint64)
P_F32 = C.POINTER(C.c_float)
P_CEX = C.POINTER(ibmc_cex)
P_SUM = C.POINTER(ibmc_check_summary)
P_OPTS = C.POINTER(ibmc_check_opts)
P_COVP = C.POINTER(ibmc_cov_params)
P_COVS = C.POINTER(ibmc_cov_summary)

# name -> (restype, argtypes); the list mirrors include/ibmc.h
SIGNATURES = {
    "ibmc_ctx_create": (I32, [I32, VP, C.POINTER(VP)]),
    "ibmc_ctx_destroy": (None, [VP]),
    "ibmc_last_error": (C.c_char_p, []),
    "ibmc_device_info": (I32, [VP, P_I32, P_I32, P_I32]),
    "ibmc_load_mlp": (I32, [VP, C.POINTER(ibmc_mlp_desc), C.POINTER(VP)]),
    "ibmc_free_mlp": (None, [VP]),
    "ibmc_check_property": (I32, [VP, VP, P_U8, I32, P_I16, I32, P_OPTS, P_SUM, P_CEX, P_CEX]),
    "ibmc_check_property_noalloc": (I32, [VP, VP, P_U8, I32, P_I16, I32, P_OPTS, P_SUM, P_CEX, P_CEX]),
    "ibmc_check_property_dev": (I32, [VP, VP, VP, I32, P_I16, I32, P_OPTS, P_SUM, P_CEX, P_CEX]),
    "ibmc_check_batch": (I32, [VP, C.POINTER(ibmc_property), I32, P_OPTS, P_SUM, P_CEX, P_CEX]),
    "ibmc_check_batch_dev": (I32, [VP, C.POINTER(ibmc_property), I32, P_OPTS, P_SUM, P_CEX, P_CEX]),
    "ibmc_abort": (I32, [VP]),
    "ibmc_decode_point": (I32, [I32, I32, I32, I64, P_I32, P_I32]),
    "ibmc_replay": (I32, [VP, VP, P_U8, P_I16, I32, P_CEX, I64, P_I32]),
    "ibmc_forward": (I32, [VP, VP, P_U8, I64, VP, P_I32]),
    "ibmc_eval_points_f32": (I32, [VP, VP, P_U8, P_I16, I32, P_I32, P_I64, I64, P_F32, P_I32, P_F32, P_I32]),
    "ibmc_coverage": (I32, [VP, VP, P_U8, P_U8, I64, I32, P_COVP, P_COVS, P_U64]),
    "ibmc_coverage_dev": (I32, [VP, VP, VP, VP, I64, I32, P_COVP, P_COVS, P_U64]),
    "ibmc_coverage_all_dev": (I32, [VP, VP, VP, VP, I64, P_COVP, P_COVS, P_U64]),
    "ibmc_coverage_from_potentials": (I32, [VP, I32, P_I32, P_I64, P_I64, I64, I32, P_COVP, P_COVS, P_U64]),
    "ibmc_proposer_create": (I32, [VP, C.c_uint64, C.POINTER(VP)]),
    "ibmc_proposer_free": (None, [VP]),
    "ibmc_proposer_get": (I32, [VP, P_F32, P_F32, P_F32, P_F32]),
    "ibmc_proposer_set": (I32, [VP, P_F32, P_F32, P_F32, P_F32]),
    "ibmc_proposer_features": (I32, [VP, VP, P_U8, I32, I32, P_I16, I32, P_F32]),
    "ibmc_proposer_grad": (I32, [VP, VP, P_F32, P_F32, I32, C.c_float, P_F32, P_F32, P_F32, P_F32, P_F32]),
    "ibmc_proposer_train": (I32, [VP, VP, P_F32, P_F32, I64, C.POINTER(ibmc_train_opts), P_F32]),
    "ibmc_proposer_score": (I32, [VP, VP, VP, P_U8, I32, I32, P_I16, I32, P_F32]),
    "ibmc_proposer_score_dev": (I32, [VP, VP, VP, VP, I32, I32, P_I16, I32, VP]),
    "ibmc_label_candidates": (I32, [VP, I32, I32, P_CEX, I64, P_F32]),
    "ibmc_count_candidates": (I32, [VP, I32, I32, P_CEX, I64, P_F32]),
    "ibmc_coverage_search": (I32, [VP, VP, P_U8, I32, P_I16, I32, I32, I32, C.POINTER(ibmc_cov_params), I32,
                                   P_CEX, P_I64, P_I32, C.POINTER(ibmc_cov_summary), P_U64]),
    "ibmc_mlp_loss_grad": (I32, [VP, VP, P_U8, P_I32, I64, P_F32, C.POINTER(C.c_double)]),
    "ibmc_fit_mlp": (I32, [VP, VP, P_U8, P_I32, I64, C.POINTER(ibmc_fit_opts), C.POINTER(VP), P_F32,
                           C.POINTER(C.c_double)]),
    "ibmc_ball_digits": (I32, [I64]),
    "ibmc_check_ball": (I32, [VP, VP, P_U8, I32, I64, P_OPTS, P_SUM, P_CEX]),
    "ibmc_check_ball_batch": (I32, [VP, C.POINTER(ibmc_ball_property), I32, P_OPTS, P_SUM, P_CEX]),
    "ibmc_check_property_ranked": (I32, [VP, VP, VP, P_U8, I32, I32, I32, P_I16, I32, P_OPTS, P_SUM, P_CEX]),
    "ibmc_autotune": (I32, [VP, VP, I32, I32, C.c_char_p, I64]),
    "ibmc_set_variant": (I32, [VP, VP, C.c_char_p]),
    "ibmc_tune_save": (I32, [VP, C.c_char_p]),
    "ibmc_tune_load": (I32, [VP, C.c_char_p, P_I32]),
    "ibmc_graph_stats": (I32, [VP, P_I64, P_I64]),
    "ibmc_chosen_variant": (I32, [VP, VP, C.c_char_p, I64]),
    "ibmc_last_kernel_time": (I32, [VP, C.POINTER(C.c_double), P_I32]),
}

_LIB = None


def lib():
    """Load libibmc.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one; importing it first makes the library bind to the
        # runtime torch uses, so torch tensors and streams stay valid.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1907_12933_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _ck(rc, allow_truncated=True):
    if rc < 0 or (rc == IBMC_W_TRUNCATED and not allow_truncated):
        msg = lib().ibmc_last_error()
        raise IbmcError(rc, msg.decode() if msg else "")
    return rc


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


# ---------------------------------------------------------------------------
# context and networks
# ---------------------------------------------------------------------------

class Context:
    """An ibmc_ctx on one device.  stream: a torch.cuda.Stream (or raw
    hipStream_t integer) to run on; None lets the library create one."""

    def __init__(self, device=0, stream=None):
        raw = None
        if stream is not None:
            raw = getattr(stream, "cuda_stream", stream)
        h = VP()
        _ck(lib().ibmc_ctx_create(int(device), VP(raw) if raw else None, C.byref(h)))
        self.handle = h
        self._keep = stream

    def close(self):
        if self.handle:
            lib().ibmc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_info(self):
        n, a, b = I32(), I32(), I32()
        _ck(lib().ibmc_device_info(self.handle, C.byref(n), C.byref(a), C.byref(b)))
        return n.value, a.value, b.value


class Mlp:
    def __init__(self, ctx: Context, net):
        """net: an inputs.QNet (int8) or inputs.FNet (float32)."""
        self.ctx = ctx
        self.dims = [int(d) for d in net.dims]
        L = len(self.dims) - 1
        is_float = not hasattr(net, "shift")
        self.act = IBMC_ACT_SIGMOID_F32 if is_float else IBMC_ACT_RELU_Q8
        if is_float:
            self._W = [np.ascontiguousarray(w, np.float32) for w in net.W]
            self._b = [np.ascontiguousarray(b, np.float32) for b in net.b]
            self._shift = np.zeros(max(L - 1, 1), np.int32)
        else:
            self._W = [np.ascontiguousarray(w, np.int8) for w in net.W]
            self._b = [np.ascontiguousarray(b, np.int32) for b in net.b]
            self._shift = np.ascontiguousarray(list(net.shift) + [0], np.int32)
        self._dims = np.ascontiguousarray(self.dims, np.int32)
        Wp = (VP * L)(*[w.ctypes.data for w in self._W])
        bp = (VP * L)(*[b.ctypes.data for b in self._b])
        d = ibmc_mlp_desc(L, _ptr(self._dims, P_I32), self.act, Wp, bp, _ptr(self._shift, P_I32))
        h = VP()
        _ck(lib().ibmc_load_mlp(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h

    @classmethod
    def _from_handle(cls, ctx, handle, dims, W, b):
        """A float network the library created (e.g. by training)."""
        self = cls.__new__(cls)
        self.ctx = ctx
        self.dims = [int(d) for d in dims]
        self.act = IBMC_ACT_SIGMOID_F32
        self._W, self._b = W, b
        self.handle = handle
        return self

    @property
    def params(self):
        """(W list, b list) as loaded (host copies)."""
        return self._W, self._b

    def close(self):
        if self.handle:
            lib().ibmc_free_mlp(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ibmc_ctx_create(device=0, stream=None) -> Context:
    return Context(device, stream)


def ibmc_load_mlp(ctx: Context, net) -> Mlp:
    return Mlp(ctx, net)


def ibmc_decode_point(n_pixels, n_deltas, k, rank):
    pix = np.zeros(max(k, 1), np.int32)
    dig = np.zeros(max(k, 1), np.int32)
    _ck(lib().ibmc_decode_point(n_pixels, n_deltas, k, int(rank), _ptr(pix, P_I32), _ptr(dig, P_I32)))
    return pix[:k].copy(), dig[:k].copy()


# ---------------------------------------------------------------------------
# check
# ---------------------------------------------------------------------------

IBMC_PROPERTY_LABEL, IBMC_PROPERTY_LITERAL = 0, 1
IBMC_SIGMOID_EXP, IBMC_SIGMOID_TABLE = 0, 1


def _opts(k_min, k_max, k_step, stop_at_first, cap, tie_cap, tie_rel, on_device=False, resume=0, budget=0,
          literal_v=None, table_sigmoid=False):
    return ibmc_check_opts(int(k_min), int(k_max), int(k_step), int(bool(stop_at_first)), int(cap), int(tie_cap),
                           float(tie_rel), int(bool(on_device)), int(resume), int(budget),
                           IBMC_PROPERTY_LITERAL if literal_v is not None else IBMC_PROPERTY_LABEL,
                           IBMC_SIGMOID_TABLE if table_sigmoid else IBMC_SIGMOID_EXP,
                           float(literal_v) if literal_v is not None else 0.0)


def summary_dict(s: ibmc_check_summary):
    n = s.n_levels
    return dict(clean_label=s.clean_label, first_unsafe_k=s.first_unsafe_k, safe_up_to_k=s.safe_up_to_k,
                levels=list(s.level_k[:n]), points=list(s.points[:n]), cex=list(s.cex[:n]),
                ties=list(s.ties[:n]), points_total=s.points_total, cex_total=s.cex_total,
                near_ties_total=s.near_ties_total, seconds=s.seconds, ttfc_seconds=s.ttfc_seconds,
                points_before_first=s.points_before_first, next_cursor=s.next_cursor)


def summary_dicts(outs, n):
    """summary_dict of each of the first n entries of a ctypes summary array, read in one pass."""
    if n == 0:
        return []
    a = np.ctypeslib.as_array(outs)[:n]
    keys = a.dtype.names
    res = []
    for row in a.tolist():
        d = dict(zip(keys, row))
        m = d["n_levels"]
        res.append(dict(clean_label=d["clean_label"], first_unsafe_k=d["first_unsafe_k"],
                        safe_up_to_k=d["safe_up_to_k"], levels=d["level_k"][:m].tolist(), points=d["points"][:m].tolist(),
                        cex=d["cex"][:m].tolist(), ties=d["ties"][:m].tolist(), points_total=d["points_total"],
                        cex_total=d["cex_total"], near_ties_total=d["near_ties_total"], seconds=d["seconds"],
                        ttfc_seconds=d["ttfc_seconds"], points_before_first=d["points_before_first"],
                        next_cursor=d["next_cursor"]))
    return res


def ibmc_check_property(ctx, net, image, deltas, k_min=1, k_max=2, k_step=1, stop_at_first=False,
                        cex_capacity=1 << 20, near_tie_capacity=0, near_tie_rel=0.0, resume_cursor=0,
                        chunk_budget=0, literal_v=None, table_sigmoid=False, _entry="ibmc_check_property"):
    """Returns (summary dict, cex records, near-tie records) as numpy structured arrays.  With
    chunk_budget the call may stop early (status IBMC_W_PARTIAL, summary next_cursor >= 0);
    resume_cursor continues such a call.  literal_v: check the threshold literal with this
    reference value; table_sigmoid: float networks evaluate the table sigmoid."""
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    cex = np.empty(max(cex_capacity, 1), CEX_DTYPE)
    ties = np.empty(max(near_tie_capacity, 1), CEX_DTYPE)
    o = _opts(k_min, k_max, k_step, stop_at_first, cex_capacity, near_tie_capacity, near_tie_rel,
              resume=resume_cursor, budget=chunk_budget, literal_v=literal_v, table_sigmoid=table_sigmoid)
    s = ibmc_check_summary()
    rc = _ck(getattr(lib(), _entry)(ctx.handle, net.handle, _ptr(image, P_U8), image.size, _ptr(D, P_I16),
                                    D.size, C.byref(o), C.byref(s), cex.ctypes.data_as(P_CEX),
                                    ties.ctypes.data_as(P_CEX)))
    sd = summary_dict(s)
    sd["status"] = rc
    nrec = min(sd["cex_total"], cex_capacity)
    ntie = min(sd["near_ties_total"], near_tie_capacity)
    return sd, cex[:nrec].copy(), ties[:ntie].copy()


def ibmc_check_property_dev(ctx, net, image, deltas, k_min=1, k_max=2, k_step=1, stop_at_first=False,
                            cex_capacity=1 << 20, near_tie_capacity=0, near_tie_rel=0.0, resume_cursor=0,
                            chunk_budget=0):
    """ibmc_check_property with the image a torch uint8 device tensor; records come back to the host."""
    D = np.ascontiguousarray(deltas, np.int16)
    cex = np.empty(max(cex_capacity, 1), CEX_DTYPE)
    ties = np.empty(max(near_tie_capacity, 1), CEX_DTYPE)
    o = _opts(k_min, k_max, k_step, stop_at_first, cex_capacity, near_tie_capacity, near_tie_rel,
              resume=resume_cursor, budget=chunk_budget)
    s = ibmc_check_summary()
    rc = _ck(lib().ibmc_check_property_dev(ctx.handle, net.handle, VP(image.data_ptr()), image.numel(),
                                           _ptr(D, P_I16), D.size, C.byref(o), C.byref(s),
                                           cex.ctypes.data_as(P_CEX), ties.ctypes.data_as(P_CEX)))
    sd = summary_dict(s)
    sd["status"] = rc
    nrec = min(sd["cex_total"], cex_capacity)
    ntie = min(sd["near_ties_total"], near_tie_capacity)
    return sd, cex[:nrec].copy(), ties[:ntie].copy()


def ibmc_check_property_noalloc(ctx, net, image, deltas, k_min=1, k_max=2, k_step=1, stop_at_first=False,
                                cex_capacity=1 << 16, near_tie_capacity=0, near_tie_rel=0.0):
    """ibmc_check_property through the entry point that allocates no device
    memory (its buffers come from the library's fixed per-device scratch)."""
    return ibmc_check_property(ctx, net, image, deltas, k_min, k_max, k_step, stop_at_first, cex_capacity,
                               near_tie_capacity, near_tie_rel, _entry="ibmc_check_property_noalloc")


def _props(props, on_device):
    arr = (ibmc_property * len(props))()
    keep = []
    for i, p in enumerate(props):
        net, image, deltas, k_min, k_max = p[:5]
        k_step = p[5] if len(p) > 5 else 1
        D = np.ascontiguousarray(deltas, np.int16)
        keep.append(D)
        if on_device:
            img_ptr = image.data_ptr()
        else:
            img = np.ascontiguousarray(image, np.uint8)
            keep.append(img)
            img_ptr = img.ctypes.data
        arr[i] = ibmc_property(net.handle.value, img_ptr, _ptr(D, P_I16), D.size, k_min, k_max, k_step)
    return arr, keep


def ibmc_check_batch(ctx, props, stop_at_first=False, cex_capacity=1 << 20, near_tie_capacity=0,
                     near_tie_rel=0.0, on_device=False, cex_buf=None, records_on_device=False, resume_cursor=0,
                     chunk_budget=0, allow_abort=False, literal_v=None, table_sigmoid=False):
    """props: list of (net, image, deltas, k_min, k_max[, k_step]); with on_device the images are
    torch device tensors (uint8).  cex_buf: optional preallocated buffer of at least cex_capacity
    records, reused across calls: a CEX_DTYPE array, or with records_on_device a torch uint8
    device tensor of CEX_DTYPE.itemsize bytes per record (the records then stay on the device).
    Returns (list of summary dicts, cex records (a view into cex_buf when given; with
    records_on_device a uint8 device tensor), near-tie records, status).  With allow_abort an
    aborted call returns its partial results with status IBMC_E_ABORTED instead of raising."""
    arr, keep = _props(props, on_device)
    n = len(props)
    outs = (ibmc_check_summary * n)()
    rsz = CEX_DTYPE.itemsize
    if records_on_device:
        import torch
        if cex_buf is None or cex_buf.numel() < cex_capacity * rsz:
            cex_buf = torch.empty(max(cex_capacity, 1) * rsz, dtype=torch.uint8, device="cuda")
        tie_dev = torch.empty(max(near_tie_capacity, 1) * rsz, dtype=torch.uint8, device="cuda")
        cex_ptr, tie_ptr = C.cast(cex_buf.data_ptr(), P_CEX), C.cast(tie_dev.data_ptr(), P_CEX)
    else:
        if cex_buf is None or len(cex_buf) < cex_capacity:
            cex_buf = np.empty(max(cex_capacity, 1), CEX_DTYPE)
        ties = np.empty(max(near_tie_capacity, 1), CEX_DTYPE)
        cex_ptr, tie_ptr = cex_buf.ctypes.data_as(P_CEX), ties.ctypes.data_as(P_CEX)
    o = _opts(0, 0, 1, stop_at_first, cex_capacity, near_tie_capacity, near_tie_rel, records_on_device,
              resume=resume_cursor, budget=chunk_budget, literal_v=literal_v, table_sigmoid=table_sigmoid)
    fn = lib().ibmc_check_batch_dev if on_device else lib().ibmc_check_batch
    rc = fn(ctx.handle, arr, n, C.byref(o), outs, cex_ptr, tie_ptr)
    if not (allow_abort and rc == IBMC_E_ABORTED):
        _ck(rc)
    sums = summary_dicts(outs, n)
    tot = min(sum(s["cex_total"] for s in sums), cex_capacity)
    ttot = min(sum(s["near_ties_total"] for s in sums), near_tie_capacity)
    del keep
    if records_on_device:
        return sums, cex_buf[:tot * rsz], tie_dev[:ttot * rsz], rc
    return sums, cex_buf[:tot], ties[:ttot].copy(), rc


def ibmc_coverage_search(ctx, net, image, deltas, k, criterion, max_tests=64, **params):
    """Greedy coverage-guided tests among the points of level k.  Returns
    (tests: cex records (k, rank, label), gains per test, coverage dict with
    'bits')."""
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    tests = np.empty(max(max_tests, 1), CEX_DTYPE)
    gains = np.zeros(max(max_tests, 1), np.int64)
    nt = I32()
    out = ibmc_cov_summary()
    widths = net.dims[1:]
    tp = sum(widths[i] * widths[i + 1] for i in range(len(widths) - 1))
    bits = np.zeros(max((tp + 63) // 64, 1), np.uint64)
    p = _covp(**params)
    _ck(lib().ibmc_coverage_search(ctx.handle, net.handle, _ptr(image, P_U8), image.size, _ptr(D, P_I16), D.size,
                                   int(k), crit, C.byref(p), int(max_tests), tests.ctypes.data_as(P_CEX),
                                   _ptr(gains, P_I64), C.byref(nt), C.byref(out), _ptr(bits, P_U64)))
    n = nt.value
    d = cov_dict(out)
    d["bits"] = bits[:(tp + 63) // 64]
    return tests[:n].copy(), gains[:n].copy(), d


# ---------------------------------------------------------------------------
# training of the float networks
# ---------------------------------------------------------------------------

def n_params(dims):
    return sum(int(dims[l]) * (int(dims[l - 1]) + 1) for l in range(1, len(dims)))


def split_theta(dims, theta):
    """Flat theta (per layer W row-major, then b) -> (W list, b list)."""
    W, b, t = [], [], 0
    for l in range(1, len(dims)):
        nw = int(dims[l]) * int(dims[l - 1])
        W.append(np.ascontiguousarray(theta[t:t + nw].reshape(dims[l], dims[l - 1]), np.float32))
        t += nw
        b.append(np.ascontiguousarray(theta[t:t + dims[l]], np.float32))
        t += int(dims[l])
    return W, b


def ibmc_mlp_loss_grad(ctx, net, images, labels):
    """(mean softmax cross-entropy, gradient over flat theta) on labelled images."""
    images = np.ascontiguousarray(images, np.uint8).reshape(-1, net.dims[0])
    labels = np.ascontiguousarray(labels, np.int32)
    if len(labels) != len(images):
        raise ValueError("one label per image")
    g = np.zeros(n_params(net.dims), np.float32)
    loss = C.c_double()
    _ck(lib().ibmc_mlp_loss_grad(ctx.handle, net.handle, _ptr(images, P_U8), _ptr(labels, P_I32), len(labels),
                                 _ptr(g, P_F32), C.byref(loss)))
    return loss.value, g


def ibmc_fit_mlp(ctx, net, images, labels, epochs=10, batch=64, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 seed=0, order=None):
    """Train a copy of a float network with mini-batch Adam.  order (optional,
    int64 [epochs][n]): the images of each epoch in order.  Returns (the
    trained Mlp, the mean loss of each epoch)."""
    images = np.ascontiguousarray(images, np.uint8).reshape(-1, net.dims[0])
    labels = np.ascontiguousarray(labels, np.int32)
    if len(labels) != len(images):
        raise ValueError("one label per image")
    n = len(labels)
    ordp = None
    if order is not None:
        order = np.ascontiguousarray(order, np.int64)
        if order.shape != (epochs, n):
            raise ValueError("order must be [epochs][n]")
        ordp = _ptr(order, P_I64)
    o = ibmc_fit_opts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed), ordp)
    theta = np.zeros(n_params(net.dims), np.float32)
    losses = np.zeros(max(int(epochs), 1), np.float64)
    h = VP()
    _ck(lib().ibmc_fit_mlp(ctx.handle, net.handle, _ptr(images, P_U8), _ptr(labels, P_I32), n, C.byref(o),
                           C.byref(h), _ptr(theta, P_F32), losses.ctypes.data_as(C.POINTER(C.c_double))))
    W, b = split_theta(net.dims, theta)
    return Mlp._from_handle(ctx, h, net.dims, W, b), losses[:int(epochs)].copy()


def ibmc_ball_digits(radius_sq):
    """Digits per pixel side of the L2-ball encoding (n_deltas = 2 * this)."""
    return int(lib().ibmc_ball_digits(int(radius_sq)))


def ball_deltas(radius_sq):
    """The implicit delta set of the L2-ball encoding: -rd..-1, 1..rd."""
    rd = ibmc_ball_digits(radius_sq)
    return np.array(list(range(-rd, 0)) + list(range(1, rd + 1)), np.int16)


def ibmc_check_ball(ctx, net, image, radius_sq, k_min=1, k_max=2, k_step=1, stop_at_first=False,
                    cex_capacity=1 << 20):
    """Check the images within squared L2 distance radius_sq of image, level k
    = support size.  Returns (summary dict, cex records)."""
    image = np.ascontiguousarray(image, np.uint8)
    cex = np.empty(max(cex_capacity, 1), CEX_DTYPE)
    o = _opts(k_min, k_max, k_step, stop_at_first, cex_capacity, 0, 0.0)
    s = ibmc_check_summary()
    rc = _ck(lib().ibmc_check_ball(ctx.handle, net.handle, _ptr(image, P_U8), image.size, int(radius_sq),
                                   C.byref(o), C.byref(s), cex.ctypes.data_as(P_CEX)))
    sd = summary_dict(s)
    sd["status"] = rc
    return sd, cex[:min(sd["cex_total"], cex_capacity)].copy()


def ibmc_check_ball_batch(ctx, props, stop_at_first=False, cex_capacity=1 << 20):
    """props: list of (net, image, radius_sq, k_min, k_max[, k_step]).  Returns
    (list of summary dicts, cex records tagged with their property)."""
    n = len(props)
    arr = (ibmc_ball_property * n)()
    keep = []
    for i, pr in enumerate(props):
        net, img, r2, kmin, kmax = pr[:5]
        img = np.ascontiguousarray(img, np.uint8)
        keep.append(img)
        arr[i] = ibmc_ball_property(net.handle, img.ctypes.data, int(r2), kmin, kmax, pr[5] if len(pr) > 5 else 1, 0)
    outs = (ibmc_check_summary * n)()
    cex = np.empty(max(cex_capacity, 1), CEX_DTYPE)
    o = _opts(0, 0, 1, stop_at_first, cex_capacity, 0, 0.0)
    _ck(lib().ibmc_check_ball_batch(ctx.handle, arr, n, C.byref(o), outs, cex.ctypes.data_as(P_CEX)))
    sums = summary_dicts(outs, n)
    del keep
    return sums, cex[:min(sum(s["cex_total"] for s in sums), cex_capacity)].copy()


def ibmc_check_batch_dev(ctx, props, **kw):
    return ibmc_check_batch(ctx, props, on_device=True, **kw)


def ibmc_replay(ctx, net, image, deltas, recs):
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    recs = np.ascontiguousarray(recs, CEX_DTYPE)
    out = np.zeros(len(recs), np.int32)
    _ck(lib().ibmc_replay(ctx.handle, net.handle, _ptr(image, P_U8), _ptr(D, P_I16), D.size,
                          recs.ctypes.data_as(P_CEX), len(recs), _ptr(out, P_I32)))
    return out


def ibmc_forward(ctx, net, images, want_potentials=True):
    images = np.ascontiguousarray(images, np.uint8).reshape(-1, net.dims[0])
    n = images.shape[0]
    U = sum(net.dims[1:])
    pdt = np.float32 if net.act == IBMC_ACT_SIGMOID_F32 else np.int32
    pots = np.zeros((n, U), pdt) if want_potentials else None
    labels = np.zeros(n, np.int32)
    _ck(lib().ibmc_forward(ctx.handle, net.handle, _ptr(images, P_U8), n,
                           pots.ctypes.data if pots is not None else None, _ptr(labels, P_I32)))
    return (pots, labels) if want_potentials else labels


def ibmc_eval_points_f32(ctx, net, image, deltas, ks, ranks):
    """Logits [n][classes], labels, margins and the clean label of listed
    points of a float network, by the float enumeration's own arithmetic."""
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    ks = np.ascontiguousarray(ks, np.int32)
    ranks = np.ascontiguousarray(ranks, np.int64)
    n = ks.size
    nc = net.dims[-1]
    logits = np.zeros((max(n, 1), nc), np.float32)
    labels = np.zeros(max(n, 1), np.int32)
    margins = np.zeros(max(n, 1), np.float32)
    clean = I32()
    _ck(lib().ibmc_eval_points_f32(ctx.handle, net.handle, _ptr(image, P_U8), _ptr(D, P_I16), D.size,
                                   _ptr(ks, P_I32), _ptr(ranks, P_I64), n, _ptr(logits, P_F32), _ptr(labels, P_I32),
                                   _ptr(margins, P_F32), C.byref(clean)))
    return logits[:n], labels[:n], margins[:n], clean.value


def ibmc_abort(ctx):
    _ck(lib().ibmc_abort(ctx.handle))


def ibmc_set_variant(ctx, net, name):
    _ck(lib().ibmc_set_variant(ctx.handle, net.handle, name.encode() if name else None))


def ibmc_tune_save(ctx, path):
    _ck(lib().ibmc_tune_save(ctx.handle, str(path).encode()))


def ibmc_tune_load(ctx, path):
    n = I32()
    _ck(lib().ibmc_tune_load(ctx.handle, str(path).encode(), C.byref(n)))
    return n.value


def ibmc_chosen_variant(ctx, net):
    buf = C.create_string_buffer(256)
    _ck(lib().ibmc_chosen_variant(ctx.handle, net.handle, buf, len(buf)))
    return buf.value.decode()


def ibmc_graph_stats(ctx):
    a, b = I64(), I64()
    _ck(lib().ibmc_graph_stats(ctx.handle, C.byref(a), C.byref(b)))
    return a.value, b.value


def ibmc_last_kernel_time(ctx):
    s = C.c_double()
    n = I32()
    _ck(lib().ibmc_last_kernel_time(ctx.handle, C.byref(s), C.byref(n)))
    return s.value, n.value


# ---------------------------------------------------------------------------
# coverage
# ---------------------------------------------------------------------------

def _covp(dist_sq_min=1, ratio_num=3, ratio_den=2, P=0.8):
    return ibmc_cov_params(int(dist_sq_min), int(ratio_num), int(ratio_den), float(P))


def cov_dict(s: ibmc_cov_summary):
    return dict(covered_pairs=s.covered_pairs, total_pairs=s.total_pairs, covered_neurons=s.covered_neurons,
                total_neurons=s.total_neurons, fraction=s.fraction, literal=bool(s.literal), seconds=s.seconds)


def _pair_words(widths):
    tp = sum(int(widths[i]) * int(widths[i + 1]) for i in range(len(widths) - 1))
    return max((tp + 63) // 64, 1), (tp + 63) // 64


def ibmc_coverage(ctx, net, x1, x2, criterion, **params):
    x1 = np.ascontiguousarray(x1, np.uint8).reshape(-1, net.dims[0])
    x2 = np.ascontiguousarray(x2, np.uint8).reshape(-1, net.dims[0])
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    alloc, words = _pair_words(net.dims[1:])
    bits = np.zeros(alloc, np.uint64)
    p = _covp(**params)
    s = ibmc_cov_summary()
    _ck(lib().ibmc_coverage(ctx.handle, net.handle, _ptr(x1, P_U8), _ptr(x2, P_U8), x1.shape[0], crit, C.byref(p),
                            C.byref(s), _ptr(bits, P_U64)))
    d = cov_dict(s)
    d["bits"] = bits[:words]
    return d


def ibmc_coverage_dev(ctx, net, x1, x2, criterion, **params):
    """x1, x2: torch uint8 device tensors [n_pairs, n_pixels]."""
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    alloc, words = _pair_words(net.dims[1:])
    bits = np.zeros(alloc, np.uint64)
    p = _covp(**params)
    s = ibmc_cov_summary()
    _ck(lib().ibmc_coverage_dev(ctx.handle, net.handle, x1.data_ptr(), x2.data_ptr(), x1.shape[0], crit,
                                C.byref(p), C.byref(s), _ptr(bits, P_U64)))
    d = cov_dict(s)
    d["bits"] = bits[:words]
    return d


def ibmc_coverage_all_dev(ctx, net, x1, x2, want_bits=True, **params):
    alloc, words = _pair_words(net.dims[1:])
    bits = np.zeros(4 * alloc, np.uint64) if want_bits else None
    p = _covp(**params)
    s = (ibmc_cov_summary * 4)()
    _ck(lib().ibmc_coverage_all_dev(ctx.handle, net.handle, x1.data_ptr(), x2.data_ptr(), x1.shape[0], C.byref(p),
                                    s, _ptr(bits, P_U64)))
    out = []
    for c in range(4):
        d = cov_dict(s[c])
        if want_bits:
            d["bits"] = bits[c * alloc:c * alloc + words]
        out.append(d)
    return out


def ibmc_coverage_from_potentials(ctx, widths, u1, u2, criterion, **params):
    widths = np.ascontiguousarray(widths, np.int32)
    u1 = np.ascontiguousarray(u1, np.int64).reshape(-1)
    u2 = np.ascontiguousarray(u2, np.int64).reshape(-1)
    U = int(widths.sum())
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    alloc, words = _pair_words(list(widths))
    bits = np.zeros(alloc, np.uint64)
    p = _covp(**params)
    s = ibmc_cov_summary()
    _ck(lib().ibmc_coverage_from_potentials(ctx.handle, len(widths), _ptr(widths, P_I32), _ptr(u1, P_I64),
                                            _ptr(u2, P_I64), u1.size // U, crit, C.byref(p), C.byref(s),
                                            _ptr(bits, P_U64)))
    d = cov_dict(s)
    d["bits"] = bits[:words]
    return d


# ---------------------------------------------------------------------------
# learned proposal network
# ---------------------------------------------------------------------------

class Proposer:
    def __init__(self, ctx, seed=0):
        self.ctx = ctx
        h = VP()
        _ck(lib().ibmc_proposer_create(ctx.handle, C.c_uint64(seed), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().ibmc_proposer_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        W1 = np.zeros((PROP_HIDDEN, PROP_FEATURES), np.float32)
        b1 = np.zeros(PROP_HIDDEN, np.float32)
        w2 = np.zeros(PROP_HIDDEN, np.float32)
        c = np.zeros(1, np.float32)
        _ck(lib().ibmc_proposer_get(self.handle, _ptr(W1, P_F32), _ptr(b1, P_F32), _ptr(w2, P_F32), _ptr(c, P_F32)))
        return W1, b1, w2, float(c[0])

    def set(self, W1, b1, w2, c):
        W1 = np.ascontiguousarray(W1, np.float32); b1 = np.ascontiguousarray(b1, np.float32)
        w2 = np.ascontiguousarray(w2, np.float32); cc = np.array([c], np.float32)
        _ck(lib().ibmc_proposer_set(self.handle, _ptr(W1, P_F32), _ptr(b1, P_F32), _ptr(w2, P_F32), _ptr(cc, P_F32)))


def ibmc_proposer_create(ctx, seed=0):
    return Proposer(ctx, seed)


def ibmc_proposer_features(ctx, net, image, rows, cols, deltas):
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    f = np.zeros((image.size * D.size, PROP_FEATURES), np.float32)
    _ck(lib().ibmc_proposer_features(ctx.handle, net.handle, _ptr(image, P_U8), rows, cols, _ptr(D, P_I16), D.size,
                                     _ptr(f, P_F32)))
    return f


def ibmc_proposer_grad(ctx, prop, features, labels, pos_weight):
    f = np.ascontiguousarray(features, np.float32)
    y = np.ascontiguousarray(labels, np.float32)
    loss = np.zeros(1, np.float32)
    gW1 = np.zeros((PROP_HIDDEN, PROP_FEATURES), np.float32)
    gb1 = np.zeros(PROP_HIDDEN, np.float32)
    gw2 = np.zeros(PROP_HIDDEN, np.float32)
    gc = np.zeros(1, np.float32)
    _ck(lib().ibmc_proposer_grad(ctx.handle, prop.handle, _ptr(f, P_F32), _ptr(y, P_F32), f.shape[0],
                                 float(pos_weight), _ptr(loss, P_F32), _ptr(gW1, P_F32), _ptr(gb1, P_F32),
                                 _ptr(gw2, P_F32), _ptr(gc, P_F32)))
    return dict(loss=float(loss[0]), W1=gW1, b1=gb1, w2=gw2, c=float(gc[0]))


def ibmc_proposer_train(ctx, prop, features, labels, epochs=20, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999,
                        eps=1e-8, pos_weight=0.0, seed=0):
    f = np.ascontiguousarray(features, np.float32)
    y = np.ascontiguousarray(labels, np.float32)
    o = ibmc_train_opts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                        float(pos_weight), C.c_uint64(seed))
    losses = np.zeros(max(epochs, 1), np.float32)
    _ck(lib().ibmc_proposer_train(ctx.handle, prop.handle, _ptr(f, P_F32), _ptr(y, P_F32), f.shape[0], C.byref(o),
                                  _ptr(losses, P_F32)))
    return losses[:epochs]


def ibmc_proposer_score(ctx, prop, net, image, rows, cols, deltas):
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    s = np.zeros(image.size * D.size, np.float32)
    _ck(lib().ibmc_proposer_score(ctx.handle, prop.handle, net.handle, _ptr(image, P_U8), rows, cols,
                                  _ptr(D, P_I16), D.size, _ptr(s, P_F32)))
    return s


def ibmc_proposer_score_dev(ctx, prop, net, image, rows, cols, deltas, scores):
    """Scores into a torch float32 device tensor of n_pixels * n_deltas, from a device image."""
    D = np.ascontiguousarray(deltas, np.int16)
    assert scores.numel() >= net.dims[0] * D.size
    _ck(lib().ibmc_proposer_score_dev(ctx.handle, prop.handle, net.handle, VP(image.data_ptr()), rows, cols,
                                      _ptr(D, P_I16), D.size, VP(scores.data_ptr())))
    return scores


def ibmc_label_candidates(ctx, n_pixels, n_deltas, recs):
    """1.0 for every (pixel, delta index) candidate that occurs in the records, else 0.0."""
    recs = np.ascontiguousarray(recs, CEX_DTYPE)
    out = np.zeros(n_pixels * n_deltas, np.float32)
    _ck(lib().ibmc_label_candidates(ctx.handle, n_pixels, n_deltas, recs.ctypes.data_as(P_CEX), len(recs),
                                    _ptr(out, P_F32)))
    return out


def ibmc_count_candidates(ctx, n_pixels, n_deltas, recs):
    """Number of records in which each (pixel, delta index) candidate occurs."""
    recs = np.ascontiguousarray(recs, CEX_DTYPE)
    out = np.zeros(n_pixels * n_deltas, np.float32)
    _ck(lib().ibmc_count_candidates(ctx.handle, n_pixels, n_deltas, recs.ctypes.data_as(P_CEX), len(recs),
                                    _ptr(out, P_F32)))
    return out


def ibmc_check_property_ranked(ctx, net, prop, image, rows, cols, deltas, k_min=1, k_max=2, stop_at_first=False,
                               cex_capacity=1 << 20):
    image = np.ascontiguousarray(image, np.uint8)
    D = np.ascontiguousarray(deltas, np.int16)
    cex = np.empty(max(cex_capacity, 1), CEX_DTYPE)
    o = _opts(k_min, k_max, 1, stop_at_first, cex_capacity, 0, 0.0)
    s = ibmc_check_summary()
    rc = _ck(lib().ibmc_check_property_ranked(ctx.handle, net.handle, prop.handle if prop is not None else None,
                                              _ptr(image, P_U8), image.size, rows, cols, _ptr(D, P_I16), D.size,
                                              C.byref(o), C.byref(s), cex.ctypes.data_as(P_CEX)))
    sd = summary_dict(s)
    sd["status"] = rc
    return sd, cex[:min(sd["cex_total"], cex_capacity)].copy()


def ibmc_autotune(ctx, net, k=2, n_deltas=6):
    buf = C.create_string_buffer(1 << 16)
    _ck(lib().ibmc_autotune(ctx.handle, net.handle, int(k), int(n_deltas), buf, len(buf)))
    return buf.value.decode()
