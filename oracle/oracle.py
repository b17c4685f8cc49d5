"""ctypes front of the C oracle (fh_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only importers.  The product package
never imports this module.

All arrays are numpy float64, C-contiguous, on the host.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", 1: "bad argument", 2: "bad degree", 3: "nodes not strictly increasing",
          4: "non-finite node", 5: "weight out of range"}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with the flags its header states; returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.fho_weights.argtypes = [dp, i64, i32, dp]
        lib.fho_eval.argtypes = [dp, dp, i64, i32, dp, dp, i64, dp, dp, dp, i32, i32]
        lib.fho_backward.argtypes = [dp, dp, i64, i32, dp, i64, dp, dp, dp, dp, dp, i32]
        lib.fho_grad_scales.argtypes = [dp, dp, i64, i32, dp, i64, dp, dp, dp, dp, dp, dp, i32]
        lib.fho_eval_deriv.argtypes = [dp, dp, i64, i32, dp, dp, i64, dp, dp, dp, i32]
        lib.fho_lebesgue_max.argtypes = [dp, i64, i32, dp, i32, i32,
                                         ctypes.POINTER(ctypes.c_int64), i64, dp, dp, i32]
        lib.fho_threads.argtypes = [i32]
        for fn in (lib.fho_weights, lib.fho_eval, lib.fho_backward, lib.fho_grad_scales,
                   lib.fho_eval_deriv, lib.fho_lebesgue_max, lib.fho_threads):
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}: {STATUS.get(code, '?')}")
        self.code = code


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def weights(nodes, d):
    x = _f64(nodes)
    w = np.empty_like(x)
    st = _load().fho_weights(_p(x), x.size, int(d), _p(w))
    if st:
        raise OracleError(st)
    return w


def evaluate(nodes, values, d, pts, w=None, lebesgue=True, scale=True, compensated=True,
             nthreads=0):
    """Returns (r, Lambda or None, S or None)."""
    x, f, t = _f64(nodes), _f64(values), _f64(pts)
    wv = None if w is None else _f64(w)
    r = np.empty_like(t)
    lam = np.empty_like(t) if lebesgue else None
    sc = np.empty_like(t) if scale else None
    st = _load().fho_eval(_p(x), _p(f), x.size, int(d), _p(wv), _p(t), t.size, _p(r), _p(lam),
                          _p(sc), int(bool(compensated)), int(nthreads))
    if st:
        raise OracleError(st)
    return r, lam, sc


def backward(nodes, values, d, pts, grad, nthreads=0):
    """Returns dict with d_values, d_points, d_weights, d_nodes (total)."""
    x, f, t, g = _f64(nodes), _f64(values), _f64(pts), _f64(grad)
    df, dw, dx = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    dp = np.empty_like(t)
    st = _load().fho_backward(_p(x), _p(f), x.size, int(d), _p(t), t.size, _p(g), _p(df),
                              _p(dp), _p(dw), _p(dx), int(nthreads))
    if st:
        raise OracleError(st)
    return {"d_values": df, "d_points": dp, "d_weights": dw, "d_nodes": dx}


def eval_deriv(nodes, values, d, pts, w=None, nthreads=0):
    """(r, r', S') at the points: values, derivatives (node formula at
    hits) and the scale of the derivative's rounding error."""
    x, f, t = _f64(nodes), _f64(values), _f64(pts)
    wp = None if w is None else _f64(w)
    r, dr, sc = np.empty_like(t), np.empty_like(t), np.empty_like(t)
    st = _load().fho_eval_deriv(_p(x), _p(f), x.size, int(d), None if wp is None else _p(wp),
                                _p(t), t.size, _p(r), _p(dr), _p(sc), int(nthreads))
    if st:
        raise OracleError(st)
    return r, dr, sc


def lebesgue_max(nodes, d, samples=256, rounds=5, w=None, intervals=None, nthreads=0):
    """Largest Lebesgue function value on every interval [x_k, x_{k+1}] by
    the grid zoom of fho_lebesgue_max, and the Lebesgue constant.

    Returns (lam[n-1], x[n-1], (Lambda_max, x_max)); the constant is the
    first largest interval value (NaN values never count); a single node
    gives (1, x_0).  With `intervals` (indices k) only those are searched,
    in that order, and the constant is taken over them."""
    x = _f64(nodes)
    wp = None if w is None else _f64(w)
    ks = None
    if intervals is not None:
        ks = np.ascontiguousarray(np.asarray(intervals, dtype=np.int64))
    k = ks.size if ks is not None else max(x.size - 1, 0)
    lam, loc = np.empty(k), np.empty(k)
    st = _load().fho_lebesgue_max(
        _p(x), x.size, int(d), None if wp is None else _p(wp), int(samples), int(rounds),
        None if ks is None else ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k,
        _p(lam), _p(loc), int(nthreads))
    if st:
        raise OracleError(st)
    if x.size == 1:
        return lam, loc, (1.0, float(x[0]))
    best, at = -np.inf, np.nan
    for v, t in zip(lam, loc):
        if v > best:
            best, at = float(v), float(t)
    if best == -np.inf:
        best = np.nan
    return lam, loc, (best, at)


def grad_scales(nodes, values, d, pts, grad, nthreads=0, parts=False):
    """Error scales of the adjoint (fho_grad_scales): (s_df, s_dx, s_dn), and
    with parts=True also (s_dw, s_dxd), the two parts of s_dn."""
    x, f, t, g = _f64(nodes), _f64(values), _f64(pts), _f64(grad)
    s_df, s_dn, s_dx = np.empty_like(x), np.empty_like(x), np.empty_like(t)
    s_dw, s_dxd = np.empty_like(x), np.empty_like(x)
    st = _load().fho_grad_scales(_p(x), _p(f), x.size, int(d), _p(t), t.size, _p(g), _p(s_df),
                                 _p(s_dx), _p(s_dn), _p(s_dw), _p(s_dxd), int(nthreads))
    if st:
        raise OracleError(st)
    if parts:
        return s_df, s_dx, s_dn, s_dw, s_dxd
    return s_df, s_dx, s_dn


def threads(nthreads=0):
    return int(_load().fho_threads(int(nthreads)))
