"""Binding of the batched vector / quaternion normalization (include/nrm.h).

normalize(x) returns the lengths r and the directions x / r of the vectors
held by x, a CUDA (HIP) float32 or float64 tensor:
  layout "aos": x has shape (n, dim), the entries of one vector adjacent;
  layout "soa": x has shape (dim, n), entry k of vector i at x[k, i];
with dim 2, 3 or 4 (quaternions).  Methods (the paper's names): "scaling"
(Normalize2D/3D/4D with the Table 2 parameters, the default), "quotient"
(Algorithm 1), "quotient_pivot" (Algorithm 2, three dimensions) and
"naive".  Argument marshalling only: every step runs in the HIP library,
which must be built (fh.FhError otherwise).
"""
import torch

from . import fh

METHODS = {"scaling": 0, "quotient": 1, "quotient_pivot": 2, "naive": 3}
LAYOUTS = {"aos": 0, "soa": 1}


def normalize(x, *, method="scaling", layout="aos", lengths=True, directions=True, r_out=None,
              dir_out=None):
    """(r, xhat): r[n] (or None) and the directions in the layout of x (or
    None)."""
    lib = fh.load()
    if not isinstance(x, torch.Tensor) or x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be a float32 or float64 tensor")
    if not x.is_cuda:
        raise ValueError("x must be a device tensor")
    if x.dim() != 2:
        raise ValueError("x must be 2-dimensional: (n, dim) for aos, (dim, n) for soa")
    lay = LAYOUTS[layout]
    dim, n = (x.shape[1], x.shape[0]) if lay == 0 else (x.shape[0], x.shape[1])
    if dim not in (2, 3, 4):
        raise ValueError("vectors must have 2, 3 or 4 entries")
    x = x.contiguous()

    def _out(t, shape, name):
        if t.dtype != x.dtype or t.device != x.device or tuple(t.shape) != tuple(shape) or \
                not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {x.dtype} tensor of shape "
                             f"{tuple(shape)} on {x.device}")
        return t

    r = None
    if lengths:
        r = torch.empty(n, dtype=x.dtype, device=x.device) if r_out is None else \
            _out(r_out, (n,), "r_out")
    xh = None
    if directions:
        xh = torch.empty_like(x) if dir_out is None else _out(dir_out, x.shape, "dir_out")
    sfx = "f32" if x.dtype == torch.float32 else "f64"
    fn = getattr(lib, f"nrm_normalize{dim}_{sfx}")
    st = fn(x.data_ptr(), n, 0 if r is None else r.data_ptr(), 0 if xh is None else xh.data_ptr(),
            lay, METHODS[method], torch.cuda.current_stream(x.device).cuda_stream)
    if st:
        raise fh.FhError(st, f"nrm_normalize{dim}_{sfx}")
    return r, xh
