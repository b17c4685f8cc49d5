"""ctypes front of the normalization oracle (nrm_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only importers.  The product package
never imports this module.

Vectors are numpy arrays of shape (n, dim), float32 or float64, on the
host; the method names follow the paper: "scaling" (Normalize2D/3D/4D with
the Table 2 parameters), "quotient" (Algorithm 1), "quotient_pivot"
(Algorithm 2, three dimensions only) and "naive".
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nrm_oracle.c")
_LIB = os.path.join(_HERE, "libnrm_oracle.so")

METHODS = {"scaling": 0, "quotient": 1, "quotient_pivot": 2, "naive": 3}

_lib = None


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle with the flags its header states; returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-shared",
               "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        for sfx in ("f32", "f64"):
            fn = getattr(lib, "nro_normalize_" + sfx)
            fn.argtypes = [i32, i32, vp, i64, vp, vp]
            fn.restype = ctypes.c_int
            getattr(lib, "nro_params_" + sfx).argtypes = [vp]
        _lib = lib
    return _lib


def normalize(x, method="scaling"):
    """(r[n], xhat[n, dim]) of the n vectors x[n, dim] (float32 or float64)."""
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.float32, np.float64) or x.ndim != 2:
        raise ValueError("x must be a (n, dim) float32 or float64 array")
    n, dim = x.shape
    r = np.empty(n, dtype=x.dtype)
    xh = np.empty_like(x)
    sfx = "f32" if x.dtype == np.float32 else "f64"
    st = getattr(_load(), "nro_normalize_" + sfx)(dim, METHODS[method], x.ctypes.data, n,
                                                  r.ctypes.data, xh.ctypes.data)
    if st:
        raise OracleError(f"nro_normalize_{sfx}: status {st}")
    return r, xh


def params(dtype):
    """(tau_min, sigma_min, tau_max, sigma_max) of the oracle for dtype."""
    p = np.empty(4, dtype=dtype)
    getattr(_load(), "nro_params_" + ("f32" if p.dtype == np.float32 else "f64"))(p.ctypes.data)
    return tuple(float(v) for v in p)
