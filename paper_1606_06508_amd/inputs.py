"""Seeded synthetic inputs for the Floater-Hormann workloads.

This module holds no interpolation arithmetic: it only draws nodes, data
values and evaluation points (and upstream gradients), so that both the
kernels and the oracle can be fed the same arrays.  Every array is numpy
float64 (int64 / int32 for the batched index arrays), C-contiguous.

Workloads (the shapes of the evaluation study this library is measured on):

  runge    n=21 equispaced nodes on [-1,1], d=3, f = 1/(1+25x^2);
           10 000 uniform points followed by the 21 nodes themselves.
  sines    n=1001 equispaced, f = sum of 8 sines (frequencies U[1,20),
           amplitudes N(0,1)), 10^6 uniform points; d swept 0..8.
  split    n=4097 jittered equispaced nodes (jitter 1e-3 of the spacing
           h=2^-11, end points fixed), d=6, f = sines; 9*10^6 uniform points
           plus 10^6 points within 1e-8 of a random node, shuffled.
  batched  4096 interpolants: n ~ U{16..2048}, equispaced or Chebyshev
           second-kind nodes (50/50), d ~ U{1..10}, f ~ N(0,1),
           m ~ U{1000..100000} uniform points each; CSR-concatenated.
  grad     n=2049 equispaced, d=4, f = sines, 10^6 uniform points,
           upstream gradient g ~ N(0,1).
  vectors  n vectors in R^2, R^3 or R^4 (binary32 or binary64) for the
           normalization of the paper: random signs and mantissas; half the
           vectors draw each component's binary exponent uniformly over the
           whole range of the format (subnormals included), the other half
           draw one exponent per vector and lower each component's by 0..3,
           so both lopsided and balanced vectors appear at every scale, up to
           the largest finite values; 1e-3 of the vectors are zero and 1e-3
           carry one NaN component.
  quats    near-unit quaternions: a uniform random unit quaternion (Shoemake's
           parametrisation by three uniforms) times 1 + U[-1e-3, 1e-3].
  lebesgue a table of node sets for Lebesgue constants: for n in
           {65, 257, 1025, 4097} and d = 0..10, equispaced nodes and
           jittered equispaced nodes (interior nodes moved by 0.3 of the
           spacing times U[-1,1]); Chebyshev second-kind nodes for d <= 3
           (larger d on these nodes has Lebesgue constants beyond 1/u).

Every generator takes the sizes as arguments, so tests draw the same recipe
at reduced sizes.
"""
import numpy as np

SEED_BASE = 1606065080

WORKLOADS = ("runge", "sines", "split", "batched", "grad", "vectors", "quats", "lebesgue")


def rng(workload: str, salt: int = 0) -> np.random.Generator:
    idx = WORKLOADS.index(workload) + 1
    return np.random.Generator(np.random.PCG64(SEED_BASE + idx + 1000 * salt))


def equispaced(n: int) -> np.ndarray:
    """x_k = (2k - (n-1)) / (n-1): one rounding, end points exactly -1 and 1,
    and x_{n-1-k} = -x_k bit-for-bit."""
    if n == 1:
        return np.zeros(1)
    k = np.arange(n, dtype=np.float64)
    return (2.0 * k - (n - 1)) / (n - 1)


def cheb2(n: int) -> np.ndarray:
    """Chebyshev points of the second kind, increasing, end points forced."""
    if n == 1:
        return np.zeros(1)
    k = np.arange(n, dtype=np.float64)
    x = -np.cos(np.pi * k / (n - 1))
    x[0], x[-1] = -1.0, 1.0
    return x


def sines_params(g: np.random.Generator, terms: int = 8):
    omega = g.uniform(1.0, 20.0, size=terms)
    amp = g.standard_normal(terms)
    return omega, amp


def sines(x: np.ndarray, omega: np.ndarray, amp: np.ndarray) -> np.ndarray:
    """f(x) = sum_j amp_j sin(omega_j x)  (zero phase)."""
    return np.sin(np.multiply.outer(x, omega)) @ amp


def runge(n: int = 21, m_random: int = 10000, salt: int = 0):
    g = rng("runge", salt)
    x = equispaced(n)
    f = 1.0 / (1.0 + 25.0 * x * x)
    pts = np.concatenate([g.uniform(-1.0, 1.0, size=m_random), x])
    return {"nodes": x, "values": f, "d": 3, "points": pts}


def sines_workload(n: int = 1001, m: int = 1_000_000, salt: int = 0):
    g = rng("sines", salt)
    x = equispaced(n)
    omega, amp = sines_params(g)
    f = sines(x, omega, amp)
    pts = g.uniform(-1.0, 1.0, size=m)
    return {"nodes": x, "values": f, "degrees": list(range(0, 9)), "points": pts}


def jittered_nodes(n: int, g: np.random.Generator, rel: float = 1e-3) -> np.ndarray:
    """Equispaced on [-1,1] with spacing h = 2/(n-1), each interior node moved
    by rel*h*xi, xi ~ U[-1,1]; end points fixed (order is preserved)."""
    h = 2.0 / (n - 1)
    xi = g.uniform(-1.0, 1.0, size=n)
    xi[0] = xi[-1] = 0.0
    k = np.arange(n, dtype=np.float64)
    x = -1.0 + k * h + rel * h * xi
    x[0], x[-1] = -1.0, 1.0
    return x


def split_workload(n: int = 4097, m: int = 10_000_000, d: int = 6, near_frac: float = 0.1,
                   near: float = 1e-8, salt: int = 0):
    g = rng("split", salt)
    x = jittered_nodes(n, g)
    omega, amp = sines_params(g)
    f = sines(x, omega, amp)
    m_near = int(round(m * near_frac))
    far = g.uniform(-1.0, 1.0, size=m - m_near)
    J = g.integers(0, n, size=m_near)
    delta = g.uniform(-near, near, size=m_near)
    close = np.clip(x[J] + delta, -1.0, 1.0)
    pts = np.concatenate([far, close])
    g.shuffle(pts)
    return {"nodes": x, "values": f, "d": d, "points": pts}


def batched_workload(count: int = 4096, n_range=(16, 2048), d_range=(1, 10),
                     m_range=(1000, 100_000), salt: int = 0):
    """CSR-concatenated instances.  Per instance, in this order: n, node
    family, d, values, m, points."""
    g = rng("batched", salt)
    ns, ds, ms, nodes, vals, pts = [], [], [], [], [], []
    for _ in range(count):
        n = int(g.integers(n_range[0], n_range[1] + 1))
        cheb = bool(g.integers(0, 2))
        d = int(g.integers(d_range[0], d_range[1] + 1))
        d = min(d, n - 1)
        f = g.standard_normal(n)
        m = int(g.integers(m_range[0], m_range[1] + 1))
        t = g.uniform(-1.0, 1.0, size=m)
        ns.append(n); ds.append(d); ms.append(m)
        nodes.append(cheb2(n) if cheb else equispaced(n))
        vals.append(f)
        pts.append(t)
    n_arr = np.array(ns, dtype=np.int64)
    m_arr = np.array(ms, dtype=np.int64)
    node_off = np.zeros(count + 1, dtype=np.int64)
    node_off[1:] = np.cumsum(n_arr)
    pt_off = np.zeros(count + 1, dtype=np.int64)
    pt_off[1:] = np.cumsum(m_arr)
    return {
        "n": n_arr, "d": np.array(ds, dtype=np.int32), "m": m_arr,
        "node_off": node_off, "pt_off": pt_off,
        "nodes": np.concatenate(nodes), "values": np.concatenate(vals),
        "points": np.concatenate(pts),
    }


def grad_workload(n: int = 2049, m: int = 1_000_000, d: int = 4, salt: int = 0):
    g = rng("grad", salt)
    x = equispaced(n)
    omega, amp = sines_params(g)
    f = sines(x, omega, amp)
    pts = g.uniform(-1.0, 1.0, size=m)
    grad = g.standard_normal(m)
    return {"nodes": x, "values": f, "d": d, "points": pts, "grad": grad}


# ------------------------------------------------------------ vectors --
def _format(dtype):
    """(lowest, highest binary exponent of a value m 2^e with m in [1, 2),
    mantissa bits) of binary32 / binary64; 2^lowest is the smallest
    subnormal."""
    return (-149, 127, 23) if np.dtype(dtype) == np.float32 else (-1074, 1023, 52)


def nrm_vectors(n: int, dim: int, dtype=np.float64, salt: int = 0, zero_frac: float = 1e-3,
                nan_frac: float = 1e-3) -> np.ndarray:
    """The vectors recipe (see the module docstring) as an (n, dim) array."""
    g = rng("vectors", salt + 100 * dim + (0 if np.dtype(dtype) == np.float64 else 50))
    lo, hi, mbits = _format(dtype)
    # mantissas exactly representable in the target format, so that
    # m 2^hi never rounds up to infinity
    mant = 1.0 + np.floor(g.random((n, dim)) * 2.0 ** mbits) / 2.0 ** mbits
    sign = np.where(g.random((n, dim)) < 0.5, -1.0, 1.0)
    balanced = g.random(n) < 0.5
    e_ind = g.integers(lo, hi + 1, size=(n, dim))
    e_com = np.clip(g.integers(lo, hi + 1, size=(n, 1)) - g.integers(0, 4, size=(n, dim)), lo, hi)
    e = np.where(balanced[:, None], e_com, e_ind)
    x = np.ldexp(sign * mant, e).astype(dtype)
    zero = g.random(n) < zero_frac
    x[zero] = 0
    nan = g.random(n) < nan_frac
    x[np.flatnonzero(nan), g.integers(0, dim, size=int(nan.sum()))] = np.nan
    return np.ascontiguousarray(x)


def near_unit_quaternions(n: int, dtype=np.float64, salt: int = 0, rel: float = 1e-3):
    """The quats recipe: unit quaternions of Shoemake's parametrisation
    (u1, u2, u3 uniform) times 1 + U[-rel, rel]."""
    g = rng("quats", salt)
    u1, u2, u3 = g.random(n), g.random(n), g.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    q *= (1.0 + g.uniform(-rel, rel, size=n))[:, None]
    return np.ascontiguousarray(q.astype(dtype))


def nrm_vectors_device(n: int, dim: int, dtype: str, device, salt: int = 0,
                       zero_frac: float = 1e-3, nan_frac: float = 1e-3):
    """The vectors recipe drawn on a torch device (for sizes the host would
    take seconds to draw): the same distribution as nrm_vectors, from
    torch's generator seeded like the host recipe (different streams)."""
    import torch
    np_dtype = np.float32 if dtype in ("f32", "float32") else np.float64
    t_dtype = torch.float32 if np_dtype == np.float32 else torch.float64
    lo, hi, mbits = _format(np_dtype)
    g = torch.Generator(device=device)
    g.manual_seed(SEED_BASE + WORKLOADS.index("vectors") + 1 + 1000 * (salt + 100 * dim))
    f64 = dict(generator=g, device=device, dtype=torch.float64)
    # the fraction is clamped: a device uniform may return exactly 1.0, and a
    # mantissa of 2 at the largest exponent would overflow
    frac = torch.floor(torch.rand((n, dim), **f64) * 2.0 ** mbits).clamp_(max=2.0 ** mbits - 1)
    mant = 1.0 + frac / 2.0 ** mbits
    del frac
    mant = torch.where(torch.rand((n, dim), **f64) < 0.5, -mant, mant)
    balanced = torch.rand(n, **f64) < 0.5
    i64 = dict(generator=g, device=device, dtype=torch.int64)
    e = torch.randint(lo, hi + 1, (n, dim), **i64)
    e_com = (torch.randint(lo, hi + 1, (n, 1), **i64) - torch.randint(0, 4, (n, dim), **i64))
    e = torch.where(balanced[:, None], e_com.clamp(lo, hi), e)
    # m 2^e as (m 2^(e - e//2)) 2^(e//2): both powers of two are normal and
    # built from their bit patterns (exact), so the only rounding is the
    # final one (into the subnormals)
    half = torch.div(e, 2, rounding_mode="floor")

    def pow2(k):
        return ((k + 1023) << 52).view(torch.float64)

    x = (mant * pow2(e - half)) * pow2(half)
    x = x.to(t_dtype)
    x[torch.rand(n, **f64) < zero_frac] = 0
    nan_rows = torch.nonzero(torch.rand(n, **f64) < nan_frac).flatten()
    cols = torch.randint(0, dim, (nan_rows.numel(),), **i64)
    x[nan_rows, cols] = float("nan")
    del mant, e, e_com, half, balanced
    return x.contiguous()


def lebesgue_workload(ns=(65, 257, 1025, 4097), ds=tuple(range(11)), rel: float = 0.3,
                      cheb_dmax: int = 3, salt: int = 0):
    """List of {"family", "n", "d", "nodes"} (see the module docstring)."""
    g = rng("lebesgue", salt)
    out = []
    for n in ns:
        jit = jittered_nodes(n, g, rel)
        for d in ds:
            if d > n - 1:
                continue
            out.append({"family": "equispaced", "n": n, "d": d, "nodes": equispaced(n)})
            out.append({"family": "jittered", "n": n, "d": d, "nodes": jit})
            if d <= cheb_dmax:
                out.append({"family": "cheb2", "n": n, "d": d, "nodes": cheb2(n)})
    return out
