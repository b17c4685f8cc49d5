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

Every generator takes the sizes as arguments, so tests draw the same recipe
at reduced sizes.
"""
import numpy as np

SEED_BASE = 1606065080

WORKLOADS = ("runge", "sines", "split", "batched", "grad")


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
