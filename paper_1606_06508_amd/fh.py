"""Thin ctypes binding of libfh.so (C ABI in include/fh.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libfh.so.  Tensors must be float64, contiguous and on a ROCm
device; calls are enqueued on torch's current stream of that device.  If the
library has not been built, every call raises FhError -- there is no CPU
fallback.
"""
import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfh.so")

FH_OK, FH_E_ARG, FH_E_DEGREE, FH_E_NODES, FH_E_NONFINITE, FH_E_RANGE = 0, 1, 2, 3, 4, 5
FH_E_WORKSPACE, FH_E_HIP, FH_E_UNSUPPORTED, FH_E_TOO_LARGE = 6, 7, 8, 9
FH_FP64, FH_FP32_SPLIT = 0, 1
FH_OP_WEIGHTS, FH_OP_EVAL, FH_OP_BACKWARD, FH_OP_LEBESGUE_MAX, FH_OP_BACKWARD_SAVED = 0, 1, 2, 3, 4
FH_MAX_NODES = 1 << 28  # largest node count of one interpolant
FH_NOALLOC_MAX_NODES = 28288  # largest node count of fh_eval_noalloc
PRECISIONS = {"fp64": FH_FP64, "split": FH_FP32_SPLIT, "fp32_split": FH_FP32_SPLIT}
FH_TUNE_BATCHED_FP64, FH_TUNE_BATCHED_SPLIT = 2, 3
# kernel families of the tuner: the two precisions of fh_eval and the two of
# the batched kernel
FAMILIES = {**PRECISIONS, "batched_fp64": FH_TUNE_BATCHED_FP64,
            "batched_split": FH_TUNE_BATCHED_SPLIT}

_lib = None
_lock = threading.Lock()


class FhError(RuntimeError):
    def __init__(self, code, where=""):
        msg = status_string(code) if _lib is not None else f"status {code}"
        super().__init__(f"{where}: {msg} (status {code})" if where else msg)
        self.code = code


def load():
    """Opens libfh.so once; raises FhError if it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise FhError(FH_E_UNSUPPORTED,
                          f"{LIB_PATH} is not built (python -m paper_1606_06508_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        sig = {
            "fh_workspace_size": ([i32, i64, i64, i32, i32], sz),
            "fh_weights": ([vp, i64, i32, vp, vp, sz, vp], ctypes.c_int),
            "fh_eval": ([vp, vp, i64, i32, vp, i64, vp, vp, vp, i32, vp, sz, vp], ctypes.c_int),
            "fh_eval_noalloc": ([vp, vp, i64, i32, vp, i64, vp, vp, vp, i32, vp], ctypes.c_int),
            "fh_lebesgue": ([vp, i64, i32, vp, i64, vp, vp, i32, vp, sz, vp], ctypes.c_int),
            "fh_prepare": ([vp, vp, i64, i32, vp, i32, vp, sz, vp], ctypes.c_int),
            "fh_prepare_many": ([vp, vp, i64, ctypes.POINTER(i32), i32, i32,
                                 ctypes.POINTER(vp), sz, vp], ctypes.c_int),
            "fh_eval_prepared": ([vp, sz, i64, i32, vp, i64, vp, vp, vp], ctypes.c_int),
            "fh_eval_prepared_many": ([ctypes.POINTER(vp), sz, i32, i64, i32, vp, i64,
                                       ctypes.POINTER(vp), ctypes.POINTER(vp), vp], ctypes.c_int),
            "fh_eval_backward": ([vp, vp, i64, i32, vp, i64, vp, vp, vp, vp, i32, vp, sz, vp],
                                 ctypes.c_int),
            "fh_eval_deriv": ([vp, vp, i64, i32, vp, i64, vp, vp, vp, i32, vp, sz, vp],
                              ctypes.c_int),
            "fh_eval_forward": ([vp, vp, i64, i32, vp, i64, vp, vp, i32, vp, sz, vp],
                                ctypes.c_int),
            "fh_eval_backward_saved": ([vp, i64, i32, vp, i64, vp, vp, vp, vp, vp, i32, vp, sz,
                                        vp], ctypes.c_int),
            "fh_lebesgue_max": ([vp, i64, i32, vp, i32, i32, vp, vp, vp, i32, vp, sz, vp],
                                ctypes.c_int),
            "fh_multi_workspace_size": ([i64, i32], sz),
            "fh_eval_multi": ([vp, vp, i64, ctypes.POINTER(i32), i32, vp, i64, vp, vp, vp, sz,
                               vp], ctypes.c_int),
            "fh_batch_create": ([ctypes.POINTER(vp), i32, ctypes.POINTER(i64),
                                 ctypes.POINTER(i32), ctypes.POINTER(i64), vp, vp, vp, vp, vp, i32,
                                 vp], ctypes.c_int),
            "fh_eval_batched": ([vp, vp], ctypes.c_int),
            "fh_batch_destroy": ([vp], ctypes.c_int),
            "fh_batch_status": ([vp, vp, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
            "fh_device_status": ([vp, vp, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
            "fh_status_string": ([i32], ctypes.c_char_p),
            "fh_variant_count": ([i32], i32),
            "fh_variant_shape": ([i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)], ctypes.c_int),
            "fh_variant_lebesgue_block": ([i32, i32], i32),
            "fh_variant_node_pairs": ([i32, i32], i32),
            "fh_variant_octets": ([i32, i32], i32),
            "fh_variant_strip_points": ([i32, i32], i64),
            "fh_batch_variant": ([vp], i32),
            "fh_batch_strip_points": ([vp], i64),
            "fh_tune_set": ([i32, i64, i64, i32], ctypes.c_int),
            "fh_tune_force": ([i32, i32], ctypes.c_int),
            "fh_tune_get": ([i32, i64, i64], i32),
        }
        for dim in (2, 3, 4):
            for sfx in ("f32", "f64"):
                sig[f"nrm_normalize{dim}_{sfx}"] = ([vp, i64, vp, vp, i32, i32, vp], ctypes.c_int)
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def status_string(code: int) -> str:
    return load().fh_status_string(int(code)).decode()


def _check(code, where):
    if code != FH_OK:
        raise FhError(code, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _f64(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 tensor on a ROCm device")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _prec(precision):
    if isinstance(precision, int):
        return precision
    try:
        return PRECISIONS[precision]
    except KeyError:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}") from None


def workspace_size(op, n, m, d, precision="fp64"):
    return int(load().fh_workspace_size(int(op), int(n), int(m), int(d), _prec(precision)))


class Workspace:
    """A 256-byte aligned device workspace that grows on demand.

    The first 256 bytes hold the device status word and are zero-filled when
    the buffer is (re)allocated; the library writes everything else before
    reading it, so the rest is left as allocated.  Calls that share a
    Workspace must be ordered on one stream."""

    def __init__(self, device=None, nbytes=0):
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.buf = None
        if nbytes:
            self.reserve(nbytes)

    def reserve(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
            self.buf[:256].zero_()
            assert self.buf.data_ptr() % 256 == 0
        return self.buf

    def status(self):
        """Synchronizes, returns and clears the sticky device status bits."""
        bits = ctypes.c_uint32(0)
        code = load().fh_device_status(_ptr(self.buf), _stream(self.device), ctypes.byref(bits))
        return code, bits.value


_default_ws = {}


def default_workspace(device) -> Workspace:
    key = torch.device(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(key)
    return _default_ws[key]


def weights(nodes, d, *, out=None, ws=None):
    """Floater-Hormann weights w_k (float64 tensor [n]) on nodes' device."""
    lib = load()
    x = _f64(nodes, "nodes")
    n = x.numel()
    w = torch.empty_like(x) if out is None else _f64(out, "out")
    ws = ws or default_workspace(x.device)
    buf = ws.reserve(workspace_size(FH_OP_WEIGHTS, n, 0, d))
    _check(lib.fh_weights(_ptr(x), n, int(d), _ptr(w), _ptr(buf), buf.numel(), _stream(x.device)),
           "fh_weights")
    return w


def evaluate(nodes, values, d, x, *, lebesgue=False, weights=None, precision="fp64", out=None,
             lambda_out=None, ws=None):
    """r(x) (and Lambda(x) if lebesgue=True) of the FH interpolant."""
    lib = load()
    xn, f, t = _f64(nodes, "nodes"), _f64(values, "values"), _f64(x, "x")
    n, m = xn.numel(), t.numel()
    if f.numel() != n:
        raise ValueError("values must have as many entries as nodes")
    if weights is not None and _f64(weights, "weights").numel() != n:
        raise ValueError("weights must have as many entries as nodes")
    prec = _prec(precision)
    r = torch.empty_like(t) if out is None else _f64(out, "out")
    lam = None
    if lebesgue:
        lam = torch.empty_like(t) if lambda_out is None else _f64(lambda_out, "lambda_out")
    ws = ws or default_workspace(t.device)
    buf = ws.reserve(workspace_size(FH_OP_EVAL, n, m, d, prec))
    _check(lib.fh_eval(_ptr(xn), _ptr(f), n, int(d), _ptr(t), m, _ptr(r), _ptr(lam), _ptr(weights),
                       prec, _ptr(buf), buf.numel(), _stream(t.device)), "fh_eval")
    return (r, lam) if lebesgue else r


def evaluate_noalloc(nodes, values, d, x, out, *, lambda_out=None, weights=None,
                     precision="fp64"):
    """fh_eval_noalloc: r(x) into `out` (and Lambda(x) into `lambda_out` if
    given) with the node table in the library's fixed device array; nothing
    is allocated, here or in the library (n <= FH_NOALLOC_MAX_NODES)."""
    lib = load()
    xn, f, t = _f64(nodes, "nodes"), _f64(values, "values"), _f64(x, "x")
    r = _f64(out, "out")
    lam = None if lambda_out is None else _f64(lambda_out, "lambda_out")
    if f.numel() != xn.numel() or r.numel() != t.numel() or \
            (lam is not None and lam.numel() != t.numel()):
        raise ValueError("values, out and lambda_out must match nodes and x in size")
    if weights is not None and _f64(weights, "weights").numel() != xn.numel():
        raise ValueError("weights must have as many entries as nodes")
    _check(lib.fh_eval_noalloc(_ptr(xn), _ptr(f), xn.numel(), int(d), _ptr(t), t.numel(), _ptr(r),
                               _ptr(lam), _ptr(weights), _prec(precision), _stream(t.device)),
           "fh_eval_noalloc")
    return r if lam is None else (r, lam)


def lebesgue(nodes, d, x, *, weights=None, precision="fp64", out=None, ws=None):
    """Lebesgue function Lambda(x) of the FH scheme."""
    lib = load()
    xn, t = _f64(nodes, "nodes"), _f64(x, "x")
    n, m = xn.numel(), t.numel()
    prec = _prec(precision)
    lam = torch.empty_like(t) if out is None else _f64(out, "out")
    ws = ws or default_workspace(t.device)
    buf = ws.reserve(workspace_size(FH_OP_EVAL, n, m, d, prec))
    _check(lib.fh_lebesgue(_ptr(xn), n, int(d), _ptr(t), m, _ptr(lam), _ptr(weights), prec,
                           _ptr(buf), buf.numel(), _stream(t.device)), "fh_lebesgue")
    return lam


def eval_deriv(nodes, values, d, x, *, want_r=True, weights=None, precision="fp64", ws=None):
    """(r, r') at the points x: the interpolant and its derivative (node
    formula at exact hits); r is None when want_r is False."""
    lib = load()
    xn, f, t = _f64(nodes, "nodes"), _f64(values, "values"), _f64(x, "x")
    n, m = xn.numel(), t.numel()
    if f.numel() != n:
        raise ValueError("values must match nodes")
    if weights is not None:
        weights = _f64(weights, "weights")
    prec = _prec(precision)
    r = torch.empty_like(t) if want_r else None
    dr = torch.empty_like(t)
    ws = ws or default_workspace(t.device)
    buf = ws.reserve(workspace_size(FH_OP_EVAL, n, m, d, prec))
    _check(lib.fh_eval_deriv(_ptr(xn), _ptr(f), n, int(d), _ptr(t), m, _ptr(r), _ptr(dr),
                             _ptr(weights), prec, _ptr(buf), buf.numel(), _stream(t.device)),
           "fh_eval_deriv")
    return r, dr


def multi_workspace_size(n, K):
    return int(load().fh_multi_workspace_size(int(n), int(K)))


def eval_multi(nodes, values, degrees, x, *, lebesgue=False, ws=None):
    """K interpolants on the same nodes and points (fh_eval_multi): values is
    a (K, n) tensor, degrees K ints; returns (r, Lambda or None), each (K, m)."""
    lib = load()
    xn, t = _f64(nodes, "nodes"), _f64(x, "x")
    f = _f64(values, "values")
    n, m = xn.numel(), t.numel()
    degs = [int(v) for v in degrees]
    K = len(degs)
    if f.dim() != 2 or f.shape[0] != K or f.shape[1] != n:
        raise ValueError("values must be (len(degrees), n)")
    r = torch.empty((K, m), dtype=torch.float64, device=t.device)
    lam = torch.empty((K, m), dtype=torch.float64, device=t.device) if lebesgue else None
    ws = ws or default_workspace(t.device)
    buf = ws.reserve(multi_workspace_size(n, K))
    d_arr = (ctypes.c_int32 * K)(*degs)
    _check(lib.fh_eval_multi(_ptr(xn), _ptr(f), n, d_arr, K, _ptr(t), m, _ptr(r), _ptr(lam),
                             _ptr(buf), buf.numel(), _stream(t.device)), "fh_eval_multi")
    return r, lam


def lebesgue_max(nodes, d, *, samples=256, rounds=5, weights=None, per_interval=True, ws=None):
    """Lebesgue constant by the grid zoom of fh_lebesgue_max: returns
    (lam[n-1], loc[n-1], best[2]) with the per-interval maxima and their
    locations (None, None when per_interval is False) and best = {the
    constant, its location}, all on the nodes' device."""
    lib = load()
    xn = _f64(nodes, "nodes")
    n = xn.numel()
    if weights is not None:
        weights = _f64(weights, "weights")
    k = max(n - 1, 0)
    lam = torch.empty(k, dtype=torch.float64, device=xn.device) if per_interval else None
    loc = torch.empty(k, dtype=torch.float64, device=xn.device) if per_interval else None
    best = torch.empty(2, dtype=torch.float64, device=xn.device)
    ws = ws or default_workspace(xn.device)
    buf = ws.reserve(workspace_size(FH_OP_LEBESGUE_MAX, n, 0, d, FH_FP64))
    _check(lib.fh_lebesgue_max(_ptr(xn), n, int(d), _ptr(weights), int(samples), int(rounds),
                               _ptr(lam), _ptr(loc), _ptr(best), FH_FP64, _ptr(buf), buf.numel(),
                               _stream(xn.device)), "fh_lebesgue_max")
    return lam, loc, best


def eval_backward(nodes, values, d, x, grad_r, *, need_values=True, need_x=True,
                  need_nodes=True, precision="fp64", ws=None):
    """Adjoint of L = sum_p grad_r[p] r(x_p): (dL/dvalues, dL/dx, dL/dnodes),
    None for the ones not requested.  dL/dnodes is the total derivative
    (through the weights as well)."""
    lib = load()
    xn, f, t, g = _f64(nodes, "nodes"), _f64(values, "values"), _f64(x, "x"), _f64(grad_r, "grad_r")
    n, m = xn.numel(), t.numel()
    if f.numel() != n or g.numel() != m:
        raise ValueError("values must match nodes and grad_r must match x")
    prec = _prec(precision)
    gv = torch.empty_like(xn) if need_values else None
    gx = torch.empty_like(t) if need_x else None
    gn = torch.empty_like(xn) if need_nodes else None
    ws = ws or default_workspace(t.device)
    buf = ws.reserve(workspace_size(FH_OP_BACKWARD, n, m, d, prec))
    _check(lib.fh_eval_backward(_ptr(xn), _ptr(f), n, int(d), _ptr(t), m, _ptr(g), _ptr(gv),
                                _ptr(gx), _ptr(gn), prec, _ptr(buf), buf.numel(),
                                _stream(t.device)), "fh_eval_backward")
    return gv, gx, gn


class Saved:
    """State of fh_eval_forward for fh_eval_backward_saved: the arguments of
    the forward, its own workspace (node table, 1/D_p, r_p and the hit data
    per point) and, when the forward formed it, the derivative r'(x_p) (dr).
    Keep it, unchanged, until the last backward."""

    def __init__(self, nodes, d, x, precision, ws, dr):
        self.nodes, self.d, self.x, self.prec, self.ws = nodes, int(d), x, precision, ws
        self.dr = dr


def eval_forward(nodes, values, d, x, *, derivative=False, precision="fp64", ws=None):
    """(r, Saved): r(x) and the state its adjoint needs (fh_eval_forward),
    kept in ws (a Workspace of its own, grown as needed; a new one when
    None).  derivative: also form r'(x) (Saved.dr), from which the backward
    takes dL/dx = grad_r r'(x) -- for callers that will want dL/dx."""
    lib = load()
    xn, f, t = _f64(nodes, "nodes"), _f64(values, "values"), _f64(x, "x")
    n, m = xn.numel(), t.numel()
    if f.numel() != n:
        raise ValueError("values must match nodes")
    prec = _prec(precision)
    r = torch.empty_like(t)
    dr = torch.empty_like(t) if derivative else None
    ws = ws or Workspace(t.device)
    buf = ws.reserve(workspace_size(FH_OP_BACKWARD_SAVED, n, m, d, prec))
    _check(lib.fh_eval_forward(_ptr(xn), _ptr(f), n, int(d), _ptr(t), m, _ptr(r), _ptr(dr),
                               prec, _ptr(buf), buf.numel(), _stream(t.device)),
           "fh_eval_forward")
    return r, Saved(xn, d, t, prec, ws, dr)


def eval_backward_saved(saved, grad_r, *, need_values=True, need_x=True, need_nodes=True):
    """Adjoint of L = sum_p grad_r[p] r(x_p) from the state of eval_forward
    (fh_eval_backward_saved): (dL/dvalues, dL/dx, dL/dnodes), None for the
    ones not requested."""
    lib = load()
    xn, t, g = saved.nodes, saved.x, _f64(grad_r, "grad_r")
    n, m = xn.numel(), t.numel()
    if g.numel() != m:
        raise ValueError("grad_r must match x")
    gv = torch.empty_like(xn) if need_values else None
    gx = torch.empty_like(t) if need_x else None
    gn = torch.empty_like(xn) if need_nodes else None
    buf = saved.ws.buf
    _check(lib.fh_eval_backward_saved(_ptr(xn), n, saved.d, _ptr(t), m, _ptr(saved.dr),
                                      _ptr(g), _ptr(gv), _ptr(gx), _ptr(gn), saved.prec,
                                      _ptr(buf), buf.numel(), _stream(t.device)),
           "fh_eval_backward_saved")
    return gv, gx, gn


class Prepared:
    """An interpolant whose node table lives in its own workspace, for
    evaluation on many point batches (fh_prepare + fh_eval_prepared).
    m_hint: the point count the workspace has room for beyond the table;
    binary64 calls with up to that many points can run the octet launch
    variants (they sort the points into the workspace), larger calls run
    the pair variant of the same shape."""

    def __init__(self, nodes, values, d, *, weights=None, precision="fp64", m_hint=0,
                 _pack=True):
        lib = load()
        self.nodes = _f64(nodes, "nodes")
        self.values = None if values is None else _f64(values, "values")
        self.n, self.d, self.prec = self.nodes.numel(), int(d), _prec(precision)
        self.device = self.nodes.device
        self.ws = Workspace(self.device, workspace_size(FH_OP_EVAL, self.n, m_hint, d, self.prec))
        if not _pack:  # filled by prepare_many
            return
        buf = self.ws.buf
        _check(lib.fh_prepare(_ptr(self.nodes), _ptr(self.values), self.n, self.d, _ptr(weights),
                              self.prec, _ptr(buf), buf.numel(), _stream(self.device)),
               "fh_prepare")

    def __call__(self, x, *, want_r=True, lebesgue=False, out=None, lambda_out=None):
        lib = load()
        t = _f64(x, "x")
        if want_r and self.values is None:
            raise ValueError("prepared without values: only the Lebesgue function is available")
        r = (torch.empty_like(t) if out is None else _f64(out, "out")) if want_r else None
        lam = None
        if lebesgue:
            lam = torch.empty_like(t) if lambda_out is None else _f64(lambda_out, "lambda_out")
        buf = self.ws.buf
        _check(lib.fh_eval_prepared(_ptr(buf), buf.numel(), self.n, self.prec, _ptr(t), t.numel(),
                                    _ptr(r), _ptr(lam), _stream(t.device)), "fh_eval_prepared")
        if want_r and lebesgue:
            return r, lam
        return r if want_r else lam


def prepare_many(nodes, values, degrees, *, m_hint=0):
    """Prepared interpolants of several degrees on the same nodes and values
    (binary64), their tables packed in one launch (fh_prepare_many): the
    same tables as Prepared(nodes, values, d) for each d."""
    lib = load()
    degrees = [int(d) for d in degrees]
    preps = [Prepared(nodes, values, d, m_hint=m_hint, _pack=False) for d in degrees]
    size = max(p.ws.buf.numel() for p in preps)
    for p in preps:
        p.ws.reserve(size)
    K = len(preps)
    ds = (ctypes.c_int32 * K)(*degrees)
    wss = (ctypes.c_void_p * K)(*[p.ws.buf.data_ptr() for p in preps])
    xn = preps[0].nodes
    _check(lib.fh_prepare_many(_ptr(xn), _ptr(preps[0].values), xn.numel(), ds, K, FH_FP64, wss,
                               size, _stream(xn.device)), "fh_prepare_many")
    return preps


def eval_many(preps, x, *, want_r=True, lebesgue=False, out=None, lambda_out=None):
    """Evaluate several prepared binary64 interpolants with the same node
    count on the same points in one launch (fh_eval_prepared_many): row c of
    the (K, m) results has the bits of preps[c](x, ...) (the launch takes the
    variant tuned for its K * m points only where it sums in the same order
    as the single call's)."""
    lib = load()
    preps = list(preps)
    K = len(preps)
    if K == 0:
        raise ValueError("no prepared interpolants")
    n = preps[0].n
    if any(p.n != n or p.prec != FH_FP64 for p in preps):
        raise ValueError("eval_many takes binary64 tables with one node count")
    if want_r and any(p.values is None for p in preps):
        raise ValueError("a table prepared without values has no r")
    t = _f64(x, "x")
    m = t.numel()

    def rows(o, name):
        if o is None:
            return torch.empty((K, m), dtype=torch.float64, device=t.device)
        o = _f64(o, name)
        if o.shape != (K, m):
            raise ValueError(f"{name} must have shape (K, m)")
        return o

    r = rows(out, "out") if want_r else None
    lam = rows(lambda_out, "lambda_out") if lebesgue else None
    wss = (ctypes.c_void_p * K)(*[p.ws.buf.data_ptr() for p in preps])
    rp = None if r is None else (ctypes.c_void_p * K)(*[r[c].data_ptr() for c in range(K)])
    lp = None if lam is None else (ctypes.c_void_p * K)(*[lam[c].data_ptr() for c in range(K)])
    # every workspace holds at least the smallest one's bytes
    _check(lib.fh_eval_prepared_many(wss, min(p.ws.buf.numel() for p in preps), K, n, FH_FP64,
                                     _ptr(t), m, rp, lp, _stream(t.device)),
           "fh_eval_prepared_many")
    if want_r and lebesgue:
        return r, lam
    return r if want_r else lam


def _family(family):
    if isinstance(family, int):
        return family
    try:
        return FAMILIES[family]
    except KeyError:
        raise ValueError(f"kernel family must be one of {sorted(FAMILIES)}") from None


def variants(precision="fp64"):
    """[(id, points_per_lane, group, node_split)] of a kernel family."""
    lib = load()
    prec = _family(precision)
    out = []
    for i in range(lib.fh_variant_count(prec)):
        p, g, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.fh_variant_shape(prec, i, ctypes.byref(p), ctypes.byref(g), ctypes.byref(s)),
               "fh_variant_shape")
        out.append((i, p.value, g.value, s.value))
    return out


def variant_lebesgue_block(precision, variant):
    """Node block length of a variant whose Lebesgue sum is taken by blocks
    (0: plain sums)."""
    u = load().fh_variant_lebesgue_block(_family(precision), int(variant))
    if u < 0:
        raise FhError(FH_E_ARG, "fh_variant_lebesgue_block")
    return u


def variant_node_pairs(precision, variant):
    """True if a binary64 variant sums its node blocks by pairs of records."""
    v = load().fh_variant_node_pairs(_family(precision), int(variant))
    if v < 0:
        raise FhError(FH_E_ARG, "fh_variant_node_pairs")
    return bool(v)


def variant_octets(precision, variant):
    """True if a binary64 variant also sums the node blocks far from a point by octets."""
    v = load().fh_variant_octets(_family(precision), int(variant))
    if v < 0:
        raise FhError(FH_E_ARG, "fh_variant_octets")
    return bool(v)


def variant_strip_points(precision, variant):
    """Points one block (single-interpolant families) or one work item
    (batched families) of a variant covers."""
    v = int(load().fh_variant_strip_points(_family(precision), int(variant)))
    if v < 0:
        raise FhError(FH_E_ARG, "fh_variant_strip_points")
    return v


def tune_force(precision, variant):
    _check(load().fh_tune_force(_family(precision), int(variant)), "fh_tune_force")


def tune_set(precision, n, m, variant):
    """Records `variant` of a kernel family for calls of shape (n, m)
    (variant -1 removes the entry)."""
    _check(load().fh_tune_set(_family(precision), int(n), int(m), int(variant)), "fh_tune_set")


def tune_get(precision, n, m):
    return int(load().fh_tune_get(_family(precision), int(n), int(m)))


class Batch:
    """Many interpolants of uneven n and d evaluated by one graph launch
    (fh_batch_create / fh_eval_batched).

    n, d, m: host integer sequences (per instance); nodes_cat, values_cat,
    x_cat: device float64 tensors concatenated in instance order (CSR).
    The output tensors are allocated here unless given; the batch keeps
    references to every tensor it was created with, which must not be
    resized or moved while the batch lives."""

    def __init__(self, n, d, m, nodes_cat, values_cat, x_cat, *, lebesgue=False,
                 want_r=True, precision="fp64", r_out=None, lambda_out=None, stream=None):
        import numpy as np
        lib = load()
        self._n = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
        self._d = np.ascontiguousarray(np.asarray(d, dtype=np.int32))
        self._m = np.ascontiguousarray(np.asarray(m, dtype=np.int64))
        if not (self._n.size == self._d.size == self._m.size):
            raise ValueError("n, d and m must have one entry per instance")
        self.nodes, self.values = _f64(nodes_cat, "nodes_cat"), _f64(values_cat, "values_cat")
        self.x = _f64(x_cat, "x_cat")
        if self.nodes.numel() != int(self._n.sum()) or self.values.numel() != self.nodes.numel():
            raise ValueError("nodes_cat / values_cat must hold sum(n) entries")
        if self.x.numel() != int(self._m.sum()):
            raise ValueError("x_cat must hold sum(m) entries")
        self.device = self.x.device
        self.r = None
        if want_r:
            self.r = torch.empty_like(self.x) if r_out is None else _f64(r_out, "r_out")
        self.lam = None
        if lebesgue:
            self.lam = torch.empty_like(self.x) if lambda_out is None else _f64(lambda_out,
                                                                                 "lambda_out")
        self._h = ctypes.c_void_p()
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        st = stream if stream is not None else _stream(self.device)
        _check(lib.fh_batch_create(ctypes.byref(self._h), int(self._n.size),
                                   self._n.ctypes.data_as(i64p), self._d.ctypes.data_as(i32p),
                                   self._m.ctypes.data_as(i64p), _ptr(self.nodes),
                                   _ptr(self.values), _ptr(self.x), _ptr(self.r), _ptr(self.lam),
                                   _prec(precision), st), "fh_batch_create")

    @property
    def variant(self):
        """The launch variant the batch runs (chosen when it was created)."""
        return int(load().fh_batch_variant(self._h))

    @property
    def strip_points(self):
        """Points of one work item of the batch's launch variant."""
        return int(load().fh_batch_strip_points(self._h))

    def __call__(self):
        _check(load().fh_eval_batched(self._h, _stream(self.device)), "fh_eval_batched")
        if self.r is not None and self.lam is not None:
            return self.r, self.lam
        return self.r if self.r is not None else self.lam

    def status(self):
        bits = ctypes.c_uint32(0)
        code = load().fh_batch_status(self._h, _stream(self.device), ctypes.byref(bits))
        return code, bits.value

    def close(self):
        if self._h:
            torch.cuda.synchronize(self.device)
            load().fh_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
