"""Autotuner for the evaluation kernels' launch variants.

Every evaluation kernel of libfh.so exists in several variants (points per
lane, node-group size of the shared reciprocal, node split across the waves
of a block; fh.variants() lists them).  tune() times every variant on
synthetic problems of the requested shapes with HIP events, keeps the
fastest per (precision, n bucket, m bucket) and records it in the library's
per-process table (fh_tune_set).  save()/load() keep the table as JSON keyed
by GPU architecture, so a tuned table can be reused without re-timing.

    python -m paper_1606_06508_amd.autotune --out tune.json [--shapes 1001x1000000 ...]

All variants compute the same quantities to the same error bound; the
tuner only chooses among them by speed.
"""
import argparse
import json
import sys

import numpy as np
import torch

from . import fh

DEFAULT_SHAPES = [(21, 10021), (1001, 1_000_000), (2049, 1_000_000), (4097, 10_000_000)]


def _problem(n, m, device, seed=0):
    g = np.random.default_rng(seed)
    k = np.arange(n, dtype=np.float64)
    nodes = (2.0 * k - (n - 1)) / max(n - 1, 1)
    vals = g.standard_normal(n)
    pts = g.uniform(-1.0, 1.0, size=m)
    t = lambda a: torch.from_numpy(a).to(device)  # noqa: E731
    return t(nodes), t(vals), t(pts)


def _warm(fn, min_ms=60.0):
    """Runs fn back to back for at least min_ms of GPU time: the clock needs
    tens of milliseconds of steady work before launch times settle."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    done, k = 0.0, 1
    while done < min_ms and k <= 4096:
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        done += e0.elapsed_time(e1)
        k *= 2


def time_variants(n, m, precision="fp64", d=4, reps=5, lebesgue=True, device="cuda:0",
                  passes=2):
    """{variant id: ms of one evaluation-kernel launch}: after a warm-up,
    `passes` rounds over all variants of `reps` launches each; the best
    round's mean per variant (rounds interleave the variants, so a drifting
    clock does not favour one of them)."""
    nodes, vals, pts = _problem(n, m, device)
    prep = fh.Prepared(nodes, vals, min(d, n - 1), precision=precision, m_hint=m)
    r = torch.empty(m, dtype=torch.float64, device=device)
    lam = torch.empty(m, dtype=torch.float64, device=device) if lebesgue else None
    out = {}
    try:
        _warm(lambda: prep(pts, lebesgue=lebesgue, out=r, lambda_out=lam))
        for _ in range(passes):
            for vid, *_ in fh.variants(precision):
                fh.tune_force(precision, vid)
                prep(pts, lebesgue=lebesgue, out=r, lambda_out=lam)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    prep(pts, lebesgue=lebesgue, out=r, lambda_out=lam)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                out[vid] = min(out.get(vid, ms), ms)
    finally:
        fh.tune_force(precision, -1)
    return out


def tune(shapes=None, precisions=("fp64", "split"), reps=5, device="cuda:0", verbose=False):
    """Times all variants per shape and installs the fastest.  Returns the
    table as a JSON-ready dict."""
    shapes = shapes or DEFAULT_SHAPES
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    table = {"arch": arch, "entries": []}
    for prec in precisions:
        for n, m in shapes:
            times = time_variants(n, m, prec, reps=reps, device=device)
            best = min(times, key=times.get)
            fh.tune_set(prec, n, m, best)
            table["entries"].append({"precision": prec, "n": n, "m": m, "variant": best,
                                     "ms": times[best],
                                     "all_ms": {str(k): v for k, v in times.items()}})
            if verbose:
                shape = dict((v[0], v[1:]) for v in fh.variants(prec))[best]
                shape += (fh.variant_lebesgue_block(prec, best),)
                print(f"[tune] {prec} n={n} m={m}: variant {best} (P,G,S,U)={shape} "
                      f"{times[best]:.4f} ms; worst {max(times.values()):.4f} ms",
                      file=sys.stderr, flush=True)
    return table


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path, device="cuda:0"):
    """Installs a saved table if it was made on the same architecture.
    Returns the number of entries installed."""
    with open(path) as f:
        table = json.load(f)
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    if table.get("arch") != arch:
        return 0
    for e in table["entries"]:
        fh.tune_set(e["precision"], e["n"], e["m"], e["variant"])
    return len(table["entries"])


def main():
    ap = argparse.ArgumentParser(description="time and record the fastest kernel variants")
    ap.add_argument("--out", default=None)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--shapes", nargs="*", default=None, help="n x m, e.g. 1001x1000000")
    ap.add_argument("--precisions", nargs="*", default=["fp64", "split"])
    args = ap.parse_args()
    shapes = None
    if args.shapes:
        shapes = [tuple(int(v) for v in s.lower().split("x")) for s in args.shapes]
    table = tune(shapes, args.precisions, args.reps, verbose=True)
    if args.out:
        save(table, args.out)
    print(json.dumps(table))


if __name__ == "__main__":
    main()
