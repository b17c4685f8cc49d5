"""Autotuner for the evaluation kernels' launch variants.

Every evaluation kernel of libfh.so exists in several variants (points per
lane, node-group size of the shared reciprocal, node split across the waves
of a block, node block of the Lebesgue sums, and for batches the passes per
work item, i.e. the strip length; fh.variants() lists them).  tune() times
every variant of the single-interpolant kernels on synthetic problems of
the requested shapes, tune_batch() every variant of the batched kernel on a
given batch (one graph launch each), both with HIP events; the fastest is
recorded per (family, n bucket, m bucket) in the library's per-process
table (fh_tune_set), which fh_eval and fh_batch_create read.  Each entry
notes whether it was timed with Lambda ("lambda"); the choice serves calls
with and without it, so r keeps the same bits either way.
save()/load() keep the table as JSON keyed by GPU architecture, so a tuned
table can be reused without re-timing -- from Python, or by the library
itself through the environment variable FH_AUTOTUNE_CACHE.

    python -m paper_1606_06508_amd.autotune --out tune.json [--shapes 1001x1000000 ...]
        [--batch]

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


def _arch(device):
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tune(shapes=None, precisions=("fp64", "split"), reps=5, device="cuda:0", verbose=False,
         lebesgue=True):
    """Times all variants per shape (with or without Lambda) and installs the
    fastest.  Returns the table as a JSON-ready dict."""
    shapes = shapes or DEFAULT_SHAPES
    table = {"arch": _arch(device), "entries": []}
    for prec in precisions:
        for n, m in shapes:
            times = time_variants(n, m, prec, reps=reps, device=device, lebesgue=lebesgue)
            best = min(times, key=times.get)
            fh.tune_set(prec, n, m, best)
            table["entries"].append({"precision": prec, "n": n, "m": m,
                                     "lambda": int(bool(lebesgue)), "variant": best,
                                     "ms": times[best],
                                     "all_ms": {str(k): v for k, v in times.items()}})
            if verbose:
                shape = dict((v[0], v[1:]) for v in fh.variants(prec))[best]
                shape += (fh.variant_lebesgue_block(prec, best),)
                print(f"[tune] {prec} n={n} m={m}: variant {best} (P,G,S,U)={shape} "
                      f"{times[best]:.4f} ms; worst {max(times.values()):.4f} ms",
                      file=sys.stderr, flush=True)
    return table


def batch_key(n):
    """(n, m) under which fh_batch_create looks a batch up: the mean node
    count (rounded up) and the total number of points."""
    n = np.asarray(n, dtype=np.int64)
    return int(-(-int(n.sum()) // n.size))


def time_batch_variants(c, precision="fp64", lebesgue=False, reps=3, passes=2,
                        device="cuda:0"):
    """{variant id: ms of one graph launch} of the batched kernel family
    `precision` on the CSR batch c (inputs.batched_workload's dict): one batch
    per variant (created with that variant forced), warmed up, then `passes`
    rounds over all variants of `reps` launches each; the best round's mean
    per variant (rounds interleave the variants)."""
    family = "batched_" + precision
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)  # noqa
    nodes, vals, pts = t(c["nodes"]), t(c["values"]), t(c["points"])
    r = torch.empty_like(pts)
    lam = torch.empty_like(pts) if lebesgue else None
    batches, out = {}, {}
    try:
        for vid, *_ in fh.variants(family):
            fh.tune_force(family, vid)
            batches[vid] = fh.Batch(c["n"], c["d"], c["m"], nodes, vals, pts, lebesgue=lebesgue,
                                    precision=precision, r_out=r, lambda_out=lam)
        fh.tune_force(family, -1)
        first = next(iter(batches.values()))
        _warm(first)
        for _ in range(passes):
            for vid, b in batches.items():
                b()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    b()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                out[vid] = min(out.get(vid, ms), ms)
    finally:
        fh.tune_force(family, -1)
        for b in batches.values():
            b.close()
    return out


def tune_batch(c, precisions=("fp64",), lebesgue=False, reps=3, device="cuda:0",
               verbose=False):
    """Times every batched variant on the batch c and installs the fastest for
    that batch's shape (family, mean n, total m): a batch created afterwards
    on the same shape runs it.  Returns the table."""
    n_key, m_key = batch_key(c["n"]), int(np.asarray(c["m"]).sum())
    table = {"arch": _arch(device), "entries": []}
    for prec in precisions:
        family = "batched_" + prec
        times = time_batch_variants(c, prec, lebesgue=lebesgue, reps=reps, device=device)
        best = min(times, key=times.get)
        fh.tune_set(family, n_key, m_key, best)
        table["entries"].append({"precision": family, "n": n_key, "m": m_key,
                                 "lambda": int(bool(lebesgue)), "variant": best,
                                 "ms": times[best],
                                 "all_ms": {str(k): v for k, v in times.items()}})
        if verbose:
            shape = dict((v[0], v[1:]) for v in fh.variants(family))[best]
            print(f"[tune] {family} {len(c['n'])} instances: variant {best} (P,G,S)={shape} "
                  f"U={fh.variant_lebesgue_block(family, best)} "
                  f"strip={fh.variant_strip_points(family, best)} {times[best]:.3f} ms; "
                  f"worst {max(times.values()):.3f} ms", file=sys.stderr, flush=True)
    return table


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path, device="cuda:0"):
    """Installs a saved table if it was made on the same architecture.
    Returns the number of entries installed."""
    with open(path) as f:
        table = json.load(f)
    if table.get("arch") != _arch(device):
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
    ap.add_argument("--batch", action="store_true",
                    help="also tune the batched kernels on the 4096-instance workload")
    args = ap.parse_args()
    shapes = None
    if args.shapes:
        shapes = [tuple(int(v) for v in s.lower().split("x")) for s in args.shapes]
    table = tune(shapes, args.precisions, args.reps, verbose=True)
    if args.batch:
        from . import inputs
        table["entries"] += tune_batch(inputs.batched_workload(), args.precisions,
                                       verbose=True)["entries"]
    if args.out:
        save(table, args.out)
    print(json.dumps(table))


if __name__ == "__main__":
    main()
