#!/usr/bin/env python3
"""Throughput of Floater-Hormann evaluation on one MI355X, in node-point
pairs per second (Gpair/s), at a stated max error against the FP64 oracle.

Workload of the headline line ("sines"): n = 1001 equispaced nodes on
[-1,1], f = sum of 8 seeded sines, 10^6 uniform points, blending degree d
swept 0..8.  One step = the weight pass and node-table packing of all nine
degrees (fh_prepare_many, one launch, each degree into its own workspace)
and the fused r + Lebesgue evaluation of all 10^6 points for every d, each
degree into its own output arrays, in one launch (fh_eval_prepared_many:
per degree the bits of an fh_eval_prepared call with the same launch
variant).  value = 9 * n * m pairs
per step / step time.  Inputs are resident in HBM before timing
starts.  Before the W warm-up steps the step runs for CLOCK_WARMUP_MS
(untimed): the GPU clock ramps up over about that long, and a small W alone
left the timed steps 3-4 % slow.

Also reported in the same JSON line:
  roofline      the evaluation kernel (the dominant kernel; one launch covers
                the nine degrees), timed live with HIP events on its launch
                stream, against the FP64 vector peak (78.6 TFLOP/s) with 7
                algorithmic flops per pair;
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample;
  max_error     parity of the timed outputs against the oracle on the sample;
  forms         the other forms of the path on their own workloads: the
                launch-bound 21-node Runge case; FP64 vs FP32-split on the
                4097-node, 10^7-point clustered workload; the batched graph
                launch over 4096 uneven interpolants (in the launch variant
                the autotuner picks for it, live) vs a per-instance fh_eval
                loop; the adjoint and the derivative
                r' on 2049 nodes and 10^6 points; normalization of 10^8
                vectors; Lebesgue constants of a node-family table; several
                interpolants on the same nodes and points in one launch.
                Each form with the CPU leg reports the oracle's rate on a
                bounded sample beside its own.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import ctypes
import hashlib
import json
import re
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1606_06508_amd import fh, inputs  # noqa: E402

FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector, published
# algorithmic flops per pair with r and Lambda: sub (delta = x - x_k), div
# (t = 1 / delta), mul (a = w t), multiply-add into N (2), add into D, add
# into L (|a|); 6 without Lambda
FLOPS_PER_PAIR_RL = 7
CLOCK_WARMUP_MS = 100.0  # untimed steps before the W warm-up steps (run_sines)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_eval_f64_sines.json")
EVAL_SRC = [os.path.join(ROOT, "paper_1606_06508_amd", "csrc", f)
            for f in ("eval_f64.hip", "pair_math.h", "octets.hip")]


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _code_only(text):
    """C/C++ source without comments and blank space, so that a record of a
    kernel's counters survives edits of its comments."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def _src_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, encoding="utf-8") as fh_:
            h.update(_code_only(fh_.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(n, m):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source or
    launch variant than the one this run uses."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("src_sha256_16") != _src_hash(EVAL_SRC):
        return None
    if rec.get("variant") != fh.tune_get("fp64", n, m):  # m: points per launch
        return None
    return rec.get("hbm_bytes_per_launch")


def _variant_info(n, m):
    """The binary64 launch variant a launch of m points on n nodes runs."""
    vid = fh.tune_get("fp64", n, m)
    shape = dict((v[0], v[1:]) for v in fh.variants("fp64"))[vid]
    return {"id": vid, "points_per_lane": shape[0], "node_split": shape[2],
            "node_block": fh.variant_lebesgue_block("fp64", vid),
            "node_pairs": fh.variant_node_pairs("fp64", vid),
            "octets": fh.variant_octets("fp64", vid)}


def run_sines(dev, steps, warmup):
    """The headline step: the node tables of all nine degrees (weights and
    packing, fh_prepare_many: one launch) and the fused r + Lambda evaluation
    of all points for every degree (fh_eval_prepared_many: one launch), each
    degree into its own workspace and output arrays, on one stream.  (One
    fh_eval_prepared launch per degree, with the same launch variant, gives
    the same bits and took 5 % longer: each launch drains its last blocks
    before the next starts.
    Packing each degree with fh_prepare just before its evaluation costs a
    launch and two dependent-launch gaps per degree; packing the next degree
    on a second stream, overlapped with the current evaluation, was measured
    slower: the cross-stream event waits cost more than they hide.)"""
    c = inputs.sines_workload()
    n, m, degrees = c["nodes"].size, c["points"].size, c["degrees"]
    nodes, vals, x = _t(c["nodes"], dev), _t(c["values"], dev), _t(c["points"], dev)
    r = torch.empty((len(degrees), m), dtype=torch.float64, device=dev)
    lam = torch.empty((len(degrees), m), dtype=torch.float64, device=dev)
    ws_bytes = fh.workspace_size(fh.FH_OP_EVAL, n, m, max(degrees))
    wss = [fh.Workspace(dev, ws_bytes) for _ in degrees]
    K = len(degrees)
    d_arr = (ctypes.c_int32 * K)(*degrees)
    ws_arr = (ctypes.c_void_p * K)(*[w.buf.data_ptr() for w in wss])
    r_arr = (ctypes.c_void_p * K)(*[r[i].data_ptr() for i in range(K)])
    l_arr = (ctypes.c_void_p * K)(*[lam[i].data_ptr() for i in range(K)])
    lib = fh.load()
    stream = torch.cuda.current_stream(dev)
    sptr = fh._stream(dev)
    P = fh._ptr

    def step(evs=None):
        st = lib.fh_prepare_many(P(nodes), P(vals), n, d_arr, K, fh.FH_FP64, ws_arr, ws_bytes, sptr)
        if evs is not None:
            evs.append(torch.cuda.Event(enable_timing=True))
            evs[-1].record(stream)
        st |= lib.fh_eval_prepared_many(ws_arr, ws_bytes, K, n, fh.FH_FP64, P(x), m, r_arr, l_arr,
                                        sptr)
        if evs is not None:
            evs.append(torch.cuda.Event(enable_timing=True))
            evs[-1].record(stream)
        if st:
            raise fh.FhError(st, "bench step")

    # the clock needs ~100 ms of steady work to ramp up: steps for that long
    # first, then the W counted warm-up steps (a small W alone left the
    # timed steps 3-4 % slow)
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < CLOCK_WARMUP_MS:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = []
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        step(evs)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    kern_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(0, len(evs), 2)]
    # outputs of the last degree (d = 8) for the parity sample
    return {
        "n": n, "m": m, "degrees": degrees, "total_ms": total_ms, "kernel_ms": kern_ms,
        "r_last": r[-1], "lam_last": lam[-1], "case": c,
    }


def cpu_baseline(case, gpu_r, gpu_lam, target_s):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload (the first m_s points, every d), plus parity on that sample for
    the last degree (whose GPU outputs are at hand)."""
    from oracle import metrics, oracle
    nodes, vals, pts = case["nodes"], case["values"], case["points"]
    n = nodes.size
    probe = pts[:4000]
    t = time.perf_counter()
    oracle.evaluate(nodes, vals, 4, probe)
    per_point = (time.perf_counter() - t) / probe.size
    m_s = int(min(pts.size, max(4000, target_s / (9 * per_point))))
    sample = pts[:m_s]
    t = time.perf_counter()
    for d in case["degrees"]:
        r_o, lam_o, s_o = oracle.evaluate(nodes, vals, d, sample)
    el = time.perf_counter() - t
    pairs = 9 * n * m_s
    stats = metrics.parity(gpu_r[:m_s], gpu_lam[:m_s], r_o, lam_o, s_o)
    # one thread on a small sample (d = 4)
    one = pts[:max(1000, min(m_s, int(1.5 / (per_point * oracle.threads()))))]
    t = time.perf_counter()
    oracle.evaluate(nodes, vals, 4, one, nthreads=1)
    el1 = time.perf_counter() - t
    base = {"value": pairs / el / 1e9, "unit": "Gpair/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"first {m_s} of the 10^6 points, all 9 degrees, n={n} "
                      f"(compensated FP64, {el:.1f} s)",
            "single_core_value": n * one.size / el1 / 1e9,
            "single_core_sample": f"first {one.size} points, d=4, one thread",
            **host_cpu()}
    return base, stats


def host_cpu():
    """CPU model and logical/physical counts of this host (/proc/cpuinfo)."""
    model, logical, cores = None, 0, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name":
                    model = model or val
                    logical += 1
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                    cores.add((phys, core))
    except OSError:
        pass
    return {"cpu_model": model, "host_logical_cpus": logical,
            "host_physical_cores": len(cores) or None}


def launch_overheads(dev, reps=200):
    """Time of an (almost) empty kernel launch and of an empty one-kernel
    graph replay on this machine: the launch cost that the per-launch figures
    contain (the analogue of subtracting an empty loop)."""
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    ms_k = _time_ms(lambda: t.add_(0.0), reps)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        t.add_(0.0)
    torch.cuda.current_stream(dev).wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        t.add_(0.0)
    ms_g = _time_ms(g.replay, reps)
    return {"empty_kernel_us": ms_k * 1e3, "empty_graph_us": ms_g * 1e3,
            "how": "1-element add_ launched, and replayed as a captured graph, "
                   f"{reps} times back to back; mean per launch"}


def run_runge_form(dev, reps, with_cpu):
    """The Runge workload (n = 21 equispaced nodes, d = 3, 10 021 points):
    one fh_eval call (weights, packing and the fused r + Lambda evaluation)
    is launch-bound -- a few microseconds of work behind two launches --
    so it is reported per call next to the empty-launch time; with_cpu adds
    the oracle's rate on the whole workload and its max error."""
    c = inputs.runge()
    n, m = c["nodes"].size, c["points"].size
    nodes, vals, x = _t(c["nodes"], dev), _t(c["values"], dev), _t(c["points"], dev)
    ws = fh.Workspace(dev, fh.workspace_size(fh.FH_OP_EVAL, n, m, c["d"]))
    r = torch.empty_like(x)
    lam = torch.empty_like(x)
    ms = _time_ms(lambda: fh.evaluate(nodes, vals, c["d"], x, lebesgue=True, out=r,
                                      lambda_out=lam, ws=ws), max(reps, 200))
    out = {"workload": f"runge: n={n} equispaced, d={c['d']}, f=1/(1+25x^2), m={m}",
           "us_per_call": ms * 1e3, "Gpair_s": n * m / (ms * 1e-3) / 1e9}
    if with_cpu:
        from oracle import metrics, oracle
        t0 = time.perf_counter()
        for _ in range(20):
            r_o, lam_o, s_o = oracle.evaluate(c["nodes"], c["values"], c["d"], c["points"])
        dt = (time.perf_counter() - t0) / 20
        out["cpu_oracle"] = {"us_per_call": dt * 1e6, "Gpair_s": n * m / dt / 1e9,
                             "cores": oracle.threads(), "sample": "the whole workload"}
        st = metrics.parity(r.cpu().numpy(), lam.cpu().numpy(), r_o, lam_o, s_o)
        out["max_error"] = {k: v for k, v in st.items() if k.startswith("e_")}
    return out


def run_split_forms(dev, reps, with_cpu):
    """FP64 vs FP32-split on the clustered 4097-node, 10^7-point workload
    (eval kernel only, node table prepared once)."""
    c = inputs.split_workload()
    n, m = c["nodes"].size, c["points"].size
    nodes, vals, x = _t(c["nodes"], dev), _t(c["values"], dev), _t(c["points"], dev)
    out = {}
    res = {}
    for prec in ("fp64", "split"):
        prep = fh.Prepared(nodes, vals, c["d"], precision=prec, m_hint=m)
        r = torch.empty(m, dtype=torch.float64, device=dev)
        lam = torch.empty(m, dtype=torch.float64, device=dev)
        ms = _time_ms(lambda: prep(x, lebesgue=True, out=r, lambda_out=lam), reps)
        out[prec] = {"Gpair_s": n * m / (ms * 1e-3) / 1e9, "ms": ms}
        res[prec] = (r, lam)
    out["split_speedup_vs_fp64"] = out["split"]["Gpair_s"] / out["fp64"]["Gpair_s"]
    if with_cpu:
        from oracle import metrics, oracle
        idx = np.random.default_rng(0).choice(m, 4000, replace=False)
        t0 = time.perf_counter()
        r_o, lam_o, s_o = oracle.evaluate(c["nodes"], c["values"], c["d"], c["points"][idx])
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"Gpair_s": n * idx.size / dt / 1e9, "cores": oracle.threads(),
                             "sample": f"{idx.size} seeded points of the workload, r and Lambda"}
        for prec in ("fp64", "split"):
            r, lam = res[prec]
            st = metrics.parity(r.cpu().numpy()[idx], lam.cpu().numpy()[idx], r_o, lam_o, s_o,
                                metrics.FP64_LAMBDA_MAX if prec == "fp64"
                                else metrics.SPLIT_LAMBDA_MAX)
            out[prec]["max_error_sample4000"] = {k: v for k, v in st.items()
                                                 if k.startswith(("e_", "n_"))}
    out["workload"] = f"split: n={n} jittered, d={c['d']}, m={m} (10% within 1e-8 of a node)"
    return out


def _warm(fn, ms=50.0):
    """Back-to-back calls of fn for about `ms` milliseconds: the clock needs
    tens of milliseconds of steady work to ramp up (more after an idle
    phase such as the host-side oracle)."""
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-6)
    for _ in range(min(int(ms * 1e-3 / one), 20000)):
        fn()
    torch.cuda.synchronize()


def _time_ms(fn, reps, stream=None):
    _warm(fn)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_batched_form(dev, reps, with_cpu, tune=True):
    """All 4096 interpolants in one graph launch (weights + evaluation of
    every instance), against a loop of one fh_eval call per instance on the
    same stream (same precision, same outputs).  With tune, the autotuner
    first times every batched launch variant on this batch (one graph launch
    each) and installs the fastest; the timed batches then run its choice."""
    from paper_1606_06508_amd import autotune
    c = inputs.batched_workload()
    n, d, m = c["n"], c["d"], c["m"]
    pairs = float((n * m).sum())
    nodes, vals, x = _t(c["nodes"], dev), _t(c["values"], dev), _t(c["points"], dev)
    out = {"workload": f"batched: {n.size} instances, n in [16,2048], d in [1,10], "
                       f"sum m = {int(m.sum())}, pairs = {pairs:.3e}"}
    r_loop = torch.empty_like(x)
    for prec in ("fp64", "split"):
        family = "batched_" + prec
        tuned = None
        if tune:
            (tuned,) = autotune.tune_batch(c, (prec,), reps=2, device=dev)["entries"]
        b = fh.Batch(n, d, m, nodes, vals, x, precision=prec)
        ms = _time_ms(b, reps)
        shape = dict((v[0], v[1:]) for v in fh.variants(family))[b.variant]
        out[prec] = {"Gpair_s": pairs / (ms * 1e-3) / 1e9, "ms_per_launch": ms,
                     "variant": {"id": b.variant, "chosen_by": "autotuner, live" if tune
                                 else "built-in table",
                                 "points_per_lane": shape[0], "node_split": shape[2],
                                 "lebesgue_block": fh.variant_lebesgue_block(family, b.variant),
                                 "strip_points": b.strip_points}}
        if tuned is not None:
            out[prec]["variant"]["tuner_ms_by_variant"] = {
                k: round(v, 3) for k, v in sorted(tuned["all_ms"].items(), key=lambda t: t[1])}
        if with_cpu:
            from oracle import metrics, oracle
            g = np.random.default_rng(1)
            worst, pairs_o, secs_o = {}, 0.0, 0.0
            for i in g.choice(n.size, 12, replace=False):
                ns = slice(int(c["node_off"][i]), int(c["node_off"][i + 1]))
                p0, p1 = int(c["pt_off"][i]), int(c["pt_off"][i + 1])
                sel = np.arange(p0, p1)[g.choice(p1 - p0, min(1000, p1 - p0), replace=False)]
                t0 = time.perf_counter()
                r_o, lam_o, s_o = oracle.evaluate(c["nodes"][ns], c["values"][ns], int(d[i]),
                                                  c["points"][sel], lebesgue=True)
                secs_o += time.perf_counter() - t0
                pairs_o += float(n[i]) * sel.size
                st = metrics.parity(b.r[torch.from_numpy(sel).to(dev)].cpu().numpy(), None, r_o,
                                    lam_o, s_o)
                for k, v in st.items():
                    if k.startswith("e_"):
                        worst[k] = max(worst.get(k, 0.0), v)
                    elif k.startswith("n_"):
                        worst[k] = worst.get(k, 0) + v
            worst["n_points"] = 12000 if n.size >= 12 else None
            out[prec]["max_error_12_instances"] = worst
            if prec == "fp64":
                out["cpu_oracle"] = {"Gpair_s": pairs_o / secs_o / 1e9, "cores": oracle.threads(),
                                     "sample": "up to 1000 seeded points of 12 seeded instances"}
        b.close()
        # the same batch with the Lebesgue function as well
        b = fh.Batch(n, d, m, nodes, vals, x, precision=prec, lebesgue=True)
        ms = _time_ms(b, reps)
        out[prec]["with_lebesgue"] = {"Gpair_s": pairs / (ms * 1e-3) / 1e9, "ms_per_launch": ms}
        b.close()
    ws = fh.Workspace(dev, fh.workspace_size(fh.FH_OP_EVAL, int(n.max()), int(m.max()), 0))
    no, po = c["node_off"], c["pt_off"]

    def loop():
        for i in range(n.size):
            fh.evaluate(nodes[no[i]:no[i + 1]], vals[no[i]:no[i + 1]], int(d[i]),
                        x[po[i]:po[i + 1]], out=r_loop[po[i]:po[i + 1]], ws=ws)

    ms_loop = _time_ms(loop, 1)
    out["per_instance_loop_fp64"] = {"Gpair_s": pairs / (ms_loop * 1e-3) / 1e9, "ms": ms_loop}
    out["batched_speedup_vs_loop_fp64"] = ms_loop / out["fp64"]["ms_per_launch"]
    out["split_batched_speedup_vs_fp64_batched"] = (out["fp64"]["ms_per_launch"]
                                                    / out["split"]["ms_per_launch"])
    return out


def run_backward_form(dev, reps, with_cpu):
    """Adjoint of sum_p g_p r(x_p) on the 2049-node, 10^6-point workload:
    gradients with respect to values, points and nodes, binary64 and
    FP32-split, and the forward derivative r'(x_p) with r(x_p); with_cpu adds
    the max scaled error of every output against the oracle's adjoint and
    derivative (|path - oracle| / sum of |terms|, see the oracle's error
    scales)."""
    c = inputs.grad_workload()
    n, m = c["nodes"].size, c["points"].size
    nodes, vals, x, g = (_t(c[k], dev) for k in ("nodes", "values", "points", "grad"))
    out = {"workload": f"grad: n={n} equispaced, d={c['d']}, m={m}, g ~ N(0,1)"}
    ref = None
    if with_cpu:
        from oracle import oracle
        t0 = time.perf_counter()
        o = oracle.backward(c["nodes"], c["values"], c["d"], c["points"], c["grad"])
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"backward_Gpair_s": n * m / dt / 1e9, "backward_s": dt,
                             "cores": oracle.threads(), "sample": "the whole workload (all gradients)"}
        sc = oracle.grad_scales(c["nodes"], c["values"], c["d"], c["points"], c["grad"])
        ref = ((o["d_values"], sc[0]), (o["d_points"], sc[1]), (o["d_nodes"], sc[2]))
        _, dr_o, s_o = oracle.eval_deriv(c["nodes"], c["values"], c["d"], c["points"])
    for prec in ("fp64", "split"):
        ws = fh.Workspace(dev, fh.workspace_size(fh.FH_OP_BACKWARD, n, m, c["d"], prec))
        ms_b = _time_ms(lambda: fh.eval_backward(nodes, vals, c["d"], x, g, precision=prec,
                                                 ws=ws), reps)
        # only some gradients: the passes and sums they need
        ms_bv = _time_ms(lambda: fh.eval_backward(nodes, vals, c["d"], x, g, need_x=False,
                                                  need_nodes=False, precision=prec, ws=ws), reps)
        ms_bx = _time_ms(lambda: fh.eval_backward(nodes, vals, c["d"], x, g, need_values=False,
                                                  need_nodes=False, precision=prec, ws=ws), reps)
        ms_f = _time_ms(lambda: fh.evaluate(nodes, vals, c["d"], x, precision=prec, ws=ws), reps)
        ms_d = _time_ms(lambda: fh.eval_deriv(nodes, vals, c["d"], x, precision=prec, ws=ws),
                        reps)
        out[prec] = {"backward_ms": ms_b, "forward_ms": ms_f, "deriv_ms": ms_d,
                     "backward_values_only_ms": ms_bv, "backward_points_only_ms": ms_bx,
                     "backward_Gpair_s": n * m / (ms_b * 1e-3) / 1e9,
                     "forward_Gpair_s": n * m / (ms_f * 1e-3) / 1e9,
                     "deriv_Gpair_s": n * m / (ms_d * 1e-3) / 1e9}
        # saved-state adjoint (the autograd path): the forward keeps 1/D, r and
        # the hit data; the backward forms each reciprocal once
        wss = fh.Workspace(dev, fh.workspace_size(fh.FH_OP_BACKWARD_SAVED, n, m, c["d"], prec))
        ms_fs = _time_ms(lambda: fh.eval_forward(nodes, vals, c["d"], x, precision=prec, ws=wss),
                         reps)
        _, st = fh.eval_forward(nodes, vals, c["d"], x, precision=prec, ws=wss)
        ms_bs = _time_ms(lambda: fh.eval_backward_saved(st, g), reps)
        ms_bsv = _time_ms(lambda: fh.eval_backward_saved(st, g, need_x=False, need_nodes=False),
                          reps)
        ms_bsx = _time_ms(lambda: fh.eval_backward_saved(st, g, need_values=False,
                                                         need_nodes=False), reps)
        # ... and with the derivative kept by the forward (dL/dx = g r')
        wsd = fh.Workspace(dev, fh.workspace_size(fh.FH_OP_BACKWARD_SAVED, n, m, c["d"], prec))
        ms_fd = _time_ms(lambda: fh.eval_forward(nodes, vals, c["d"], x, derivative=True,
                                                 precision=prec, ws=wsd), reps)
        _, std = fh.eval_forward(nodes, vals, c["d"], x, derivative=True, precision=prec,
                                 ws=wsd)
        ms_bd = _time_ms(lambda: fh.eval_backward_saved(std, g), reps)
        ms_bdx = _time_ms(lambda: fh.eval_backward_saved(std, g, need_values=False,
                                                         need_nodes=False), reps)
        out[prec]["saved_state"] = {
            "forward_ms": ms_fs, "backward_ms": ms_bs, "backward_values_only_ms": ms_bsv,
            "backward_points_only_ms": ms_bsx,
            "backward_over_forward": ms_bs / ms_fs,
            "step_ms": ms_fs + ms_bs, "step_ms_without_state": ms_f + ms_b,
            "with_derivative": {"forward_ms": ms_fd, "backward_ms": ms_bd,
                                "backward_points_only_ms": ms_bdx,
                                "backward_over_forward": ms_bd / ms_fd,
                                "step_ms": ms_fd + ms_bd}}
        if ref is not None:
            got = fh.eval_backward(nodes, vals, c["d"], x, g, precision=prec, ws=ws)
            out[prec]["max_scaled_error"] = {
                name: float(np.max(np.abs(t.cpu().numpy() - r) / np.maximum(s, 1e-300)))
                for name, t, (r, s) in zip(("dvalues", "dpoints", "dnodes"), got, ref)}
            _, dr = fh.eval_deriv(nodes, vals, c["d"], x, precision=prec, ws=ws)
            out[prec]["max_scaled_error"]["deriv"] = float(
                np.max(np.abs(dr.cpu().numpy() - dr_o) / np.maximum(s_o, 1e-300)))
            for key, state in (("max_scaled_error", st), ("max_scaled_error_with_derivative", std)):
                got = fh.eval_backward_saved(state, g)
                out[prec]["saved_state"][key] = {
                    name: float(np.max(np.abs(t.cpu().numpy() - r) / np.maximum(s, 1e-300)))
                    for name, t, (r, s) in zip(("dvalues", "dpoints", "dnodes"), got, ref)}
    out["split_backward_speedup_vs_fp64"] = out["fp64"]["backward_ms"] / out["split"]["backward_ms"]
    return out


def run_multi_form(dev, reps, with_cpu):
    """Several interpolants on the same nodes and points in one launch
    (fh_eval_multi), against one fh_eval per interpolant on the same stream:
    the headline's sweep over d = 0..8 (separate weights, r and Lambda), and
    vector-valued data (16 value columns, d = 4, shared weights).  Both
    sides produce the same bits (the multi kernel runs the per-pair
    operations of single-kernel variant 3), which with_cpu checks."""
    c = inputs.sines_workload()
    n, m = c["nodes"].size, c["points"].size
    nodes, x = _t(c["nodes"], dev), _t(c["points"], dev)
    out = {"workload": f"multi: sines nodes n={n}, m={m} points"}
    g = np.random.default_rng(7)
    cases = {"degree_sweep_0_8": (np.tile(c["values"], (9, 1)), list(range(9)), True),
             "vector_valued_16_d4": (g.standard_normal((16, n)), [4] * 16, False)}
    for name, (vals, degs, lebesgue) in cases.items():
        K = len(degs)
        v = _t(vals, dev)
        ws = fh.Workspace(dev, fh.multi_workspace_size(n, K))
        ms = _time_ms(lambda: fh.eval_multi(nodes, v, degs, x, lebesgue=lebesgue, ws=ws), reps)
        ws1 = fh.Workspace(dev, fh.workspace_size(fh.FH_OP_EVAL, n, m, max(degs)))
        outs = [torch.empty_like(x) for _ in range(K)]
        lams = [torch.empty_like(x) for _ in range(K)] if lebesgue else [None] * K

        def loop():
            for k in range(K):
                fh.evaluate(nodes, v[k], degs[k], x, lebesgue=lebesgue, ws=ws1, out=outs[k],
                            lambda_out=lams[k])

        ms_loop = _time_ms(loop, reps)
        pairs = K * n * m
        out[name] = {"K": K, "lebesgue": lebesgue, "ms": ms, "Gpair_s": pairs / (ms * 1e-3) / 1e9,
                     "one_call_per_interpolant_ms": ms_loop,
                     "one_call_per_interpolant_Gpair_s": pairs / (ms_loop * 1e-3) / 1e9,
                     "speedup": ms_loop / ms}
        if with_cpu:
            r, lam = fh.eval_multi(nodes, v, degs, x, lebesgue=lebesgue, ws=ws)
            fh.tune_force("fp64", 3)
            try:
                same = all(torch.equal(r[k], fh.evaluate(nodes, v[k], degs[k], x)) for k in (0, K - 1))
            finally:
                fh.tune_force("fp64", -1)
            out[name]["bitwise_equal_to_single_variant_3"] = bool(same)
    return out


FLOPS_PER_PAIR_L = 5  # sub, div, mul (a = w t), add (D), add (L)


def run_lebesgue_form(dev, reps, with_cpu):
    """Lebesgue constants of the node-family table (fh_lebesgue_max, 256
    samples per round, 5 rounds): equispaced and jittered nodes for
    n in {65, 257, 1025, 4097} and d = 0..10, Chebyshev second-kind nodes
    for d <= 3.  A step computes all 104 constants (weights, per-interval
    searches, the maximum) one call after another on one stream; the
    largest configuration is also timed alone.  with_cpu adds the oracle's
    rate on sampled intervals of that configuration and the max scaled
    difference (|GPU - oracle| / (1e-13 Lambda (1 + Lambda))) on them."""
    table = inputs.lebesgue_workload()
    S, R = 256, 5
    nodes = [_t(c["nodes"], dev) for c in table]
    ws = fh.Workspace(dev, max(fh.workspace_size(fh.FH_OP_LEBESGUE_MAX, c["n"], 0, c["d"])
                               for c in table))
    pairs = float(sum((c["n"] - 1) * c["n"] for c in table)) * S * R
    res = [None] * len(table)

    def step():
        for i, c in enumerate(table):
            res[i] = fh.lebesgue_max(nodes[i], c["d"], samples=S, rounds=R, ws=ws)

    ms = _time_ms(step, reps)
    out = {"workload": f"lebesgue: {len(table)} (family, n, d) node sets, n in 65..4097, "
                       f"d in 0..10, {S} samples x {R} rounds per interval",
           "ms_all_tables": ms, "ms_per_table_mean": ms / len(table),
           "Gpair_s": pairs / (ms * 1e-3) / 1e9, "pairs": pairs}
    big = max(range(len(table)), key=lambda i: (table[i]["n"], table[i]["d"] == 3))
    cb = table[big]
    pb = float((cb["n"] - 1) * cb["n"]) * S * R
    ms_b = _time_ms(lambda: fh.lebesgue_max(nodes[big], cb["d"], samples=S, rounds=R, ws=ws),
                    reps)
    out["largest"] = {"config": f"{cb['family']} n={cb['n']} d={cb['d']}", "ms": ms_b,
                      "Gpair_s": pb / (ms_b * 1e-3) / 1e9,
                      "TFLOP_s": FLOPS_PER_PAIR_L * pb / (ms_b * 1e-3) / 1e12}
    step()
    torch.cuda.synchronize()
    consts = {}
    for c, (_, _, best) in zip(table, res):
        consts.setdefault(f"{c['family']} n={c['n']}", []).append(round(float(best[0]), 6))
    out["constants_by_d"] = consts
    if with_cpu:
        from oracle import oracle
        ks = np.random.default_rng(0).choice(cb["n"] - 1, 128, replace=False)
        t0 = time.perf_counter()
        lam_o, _, _ = oracle.lebesgue_max(cb["nodes"], cb["d"], S, R, intervals=ks)
        dt = time.perf_counter() - t0
        lam_g = res[big][0].cpu().numpy()[ks]
        out["cpu_oracle"] = {"Gpair_s": ks.size * cb["n"] * S * R / dt / 1e9,
                             "cores": oracle.threads(), "sample": f"128 intervals of {out['largest']['config']}"}
        out["max_scaled_diff_vs_oracle"] = float(np.max(
            np.abs(lam_g - lam_o) / (1e-13 * lam_o * (1 + lam_o))))
    return out


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def run_normalize_form(dev, reps, with_cpu):
    """Batched normalization (the paper's method): 10^8 vectors per kind
    (2D, 3D, quaternion; binary32 and binary64), array-of-structs, drawn on
    the device by the vectors recipe.  Per kind: vectors/s and HBM GB/s of
    the scaling algorithm (algorithmic bytes: dim entries in, dim + 1 out),
    the struct-of-arrays layout, the quotient algorithms and the naive
    formula, with the time ratios of the paper's Tables 3 and 4; the
    near-unit quaternion workload; with_cpu adds the sampled bit-for-bit
    check against the oracle and the oracle's own rate on the host."""
    from paper_1606_06508_amd.normalize import normalize
    n = 10 ** 8
    out = {"workload": f"normalize: n={n} vectors per kind, exponents over the whole range, "
                       "1e-3 zero and 1e-3 NaN vectors; plus near-unit quaternions"}
    for sfx in ("f32", "f64"):
        for dim in (2, 3, 4):
            x = inputs.nrm_vectors_device(n, dim, sfx, dev)
            esize = x.element_size()
            nbytes = n * (2 * dim + 1) * esize
            r = torch.empty(n, dtype=x.dtype, device=dev)
            xh = torch.empty_like(x)
            rec = {}
            methods = ["scaling", "quotient", "naive"] + (["quotient_pivot"] if dim == 3 else [])
            for method in methods:
                ms = _time_ms(lambda: normalize(x, method=method, r_out=r, dir_out=xh), reps)
                rec[method] = {"ms": ms, "Gvec_s": n / (ms * 1e-3) / 1e9}
            ms_s = rec["scaling"]["ms"]
            rec["scaling"]["GB_s"] = nbytes / (ms_s * 1e-3) / 1e9
            rec["scaling"]["hbm_frac"] = rec["scaling"]["GB_s"] / HBM_PEAK_GBS
            xs = x.t().contiguous()
            hs = torch.empty_like(xs)
            ms_soa = _time_ms(lambda: normalize(xs, layout="soa", r_out=r, dir_out=hs), reps)
            rec["scaling_soa"] = {"ms": ms_soa, "Gvec_s": n / (ms_soa * 1e-3) / 1e9,
                                  "GB_s": nbytes / (ms_soa * 1e-3) / 1e9}
            del xs, hs
            # practical ceiling: a plain device copy of the input array
            ms_c = _time_ms(lambda: xh.copy_(x), reps)
            rec["copy_reference"] = {"ms": ms_c,
                                     "GB_s": 2 * n * dim * esize / (ms_c * 1e-3) / 1e9}
            rec["table3_quotient_over_scaling"] = rec["quotient"]["ms"] / ms_s
            if dim == 3:
                rec["table3_pivot_over_scaling"] = rec["quotient_pivot"]["ms"] / ms_s
            rec["table4_scaling_over_naive"] = ms_s / rec["naive"]["ms"]
            if with_cpu:
                from oracle import nrm
                normalize(x, r_out=r, dir_out=xh)
                idx = torch.from_numpy(np.random.default_rng(dim).choice(n, 20000, replace=False)).to(dev)
                r_o, xh_o = nrm.normalize(x[idx].cpu().numpy(), "scaling")
                got_r, got_x = r[idx].cpu().numpy(), xh[idx].cpu().numpy()
                bad = 0
                for a, b in ((got_r, r_o), (got_x, xh_o)):
                    na, nb = np.isnan(a), np.isnan(b)
                    bad += int(np.count_nonzero(na != nb))
                    both = ~na & ~nb
                    bad += int(np.count_nonzero(a[both].view(np.uint8).reshape(-1, esize)
                                                != b[both].view(np.uint8).reshape(-1, esize)))
                rec["bitwise_mismatches_20000_sampled"] = bad
            out[f"{dim}d_{sfx}"] = rec
            del x, r, xh
            torch.cuda.empty_cache()
    for sfx, dt in (("f32", np.float32), ("f64", np.float64)):
        q = torch.from_numpy(inputs.near_unit_quaternions(10 ** 7, dt)).to(dev)
        r = torch.empty(q.shape[0], dtype=q.dtype, device=dev)
        qh = torch.empty_like(q)
        ms_s = _time_ms(lambda: normalize(q, r_out=r, dir_out=qh), reps)
        ms_n = _time_ms(lambda: normalize(q, method="naive", r_out=r, dir_out=qh), reps)
        out[f"near_unit_quaternions_{sfx}"] = {"n": q.shape[0], "scaling_ms": ms_s,
                                               "naive_ms": ms_n,
                                               "table4_scaling_over_naive": ms_s / ms_n}
    if with_cpu:
        from oracle import nrm
        xc = inputs.nrm_vectors(2 * 10 ** 6, 3, np.float64)
        t0 = time.perf_counter()
        nrm.normalize(xc, "scaling")
        dt_c = time.perf_counter() - t0
        out["cpu_oracle_3d_f64"] = {"Gvec_s": xc.shape[0] / dt_c / 1e9, "cores": 1,
                                    "sample": "2e6 vectors of the vectors recipe, scaling"}
    return out


def copy_calibration():
    """Three copies of 2^27 float64 (1 GiB read + 1 GiB written each)."""
    dev = torch.device("cuda:0")
    src = torch.rand(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                      "dispatches": 3}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # 25 untimed steps (~60 ms): the kernel time settles only after ~30 ms
    # of back-to-back work (clock ramp), 290 us -> 225 us per launch
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched form: run the built-in variant choice instead of tuning live")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (the reference dispatch that "
                         "scales the HBM byte counters)")
    ap.add_argument("--profile-form", choices=("runge", "split", "batched", "grad", "normalize",
                                               "lebesgue", "multi"),
                    help="only run one secondary form's timed loops (--steps repetitions, "
                         "no CPU work), for kernel profiles")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_form:
        dev = torch.device("cuda:0")
        run = {"runge": run_runge_form, "split": run_split_forms,
               "batched": lambda dev, reps, cpu: run_batched_form(dev, reps, cpu, tune=False),
               "grad": run_backward_form, "normalize": run_normalize_form,
               "lebesgue": run_lebesgue_form, "multi": run_multi_form}[args.profile_form]
        print(json.dumps({args.profile_form: run(dev, args.steps, False)}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(every interpolant is evaluated by one GPU; nothing is exchanged between GPUs).",
              file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    print(f"[bench] sines workload, steps={args.steps} warmup={args.warmup}", file=sys.stderr,
          flush=True)
    res = run_sines(dev, args.steps, args.warmup)
    n, m = res["n"], res["m"]
    pairs_step = len(res["degrees"]) * n * m
    ms_step = res["total_ms"] / args.steps
    value = pairs_step / (ms_step * 1e-3) / 1e9
    k_ms = float(np.mean(res["kernel_ms"]))  # one launch: all nine degrees
    achieved = FLOPS_PER_PAIR_RL * pairs_step / (k_ms * 1e-3) / 1e12
    line = {
        "metric": "node-point pairs/sec (Gpair/s) FP64 vs FP32-split vs batched at stated max error",
        "value": value, "unit": "Gpair/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "clock_warmup_ms": CLOCK_WARMUP_MS, "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sines: n=1001 equispaced, f=sum of 8 seeded sines, "
                               "m=1e6 uniform points, d=0..8, r and Lebesgue function",
                   "n": n, "m": m, "degrees": "0..8", "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(n, len(res["degrees"]) * m),
                     "kernel": "k_eval_f64_many (fused r + Lebesgue, FP64, nine degrees "
                               "per launch)",
                     "kernel_ms_avg": k_ms,
                     "kernel_Gpair_s": pairs_step / (k_ms * 1e-3) / 1e9,
                     "launch_variant": _variant_info(n, len(res["degrees"]) * m)},
    }
    print(f"[bench] sines done: {value:.1f} Gpair/s, kernel {k_ms:.3f} ms", file=sys.stderr,
          flush=True)
    if not args.no_cpu_baseline:
        base, stats = cpu_baseline(res["case"], res["r_last"].cpu().numpy(),
                                   res["lam_last"].cpu().numpy(), args.cpu_seconds)
        line["cpu_baseline"] = base
        line["max_error"] = {"vs": "FP64 oracle on the CPU-baseline sample, d=8",
                             **{k: v for k, v in stats.items() if k.startswith("e_")}}
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    line["launch_overheads"] = launch_overheads(dev)
    if not args.no_forms:
        forms = {"runge": run_runge_form(dev, 200, not args.no_cpu_baseline)}
        print("[bench] runge form done", file=sys.stderr, flush=True)
        forms["split_workload"] = run_split_forms(dev, 5, not args.no_cpu_baseline)
        print("[bench] split form done", file=sys.stderr, flush=True)
        forms["batched_workload"] = run_batched_form(dev, 3, not args.no_cpu_baseline,
                                                     tune=not args.no_tune)
        print("[bench] batched form done", file=sys.stderr, flush=True)
        forms["grad_workload"] = run_backward_form(dev, 5, not args.no_cpu_baseline)
        print("[bench] backward form done", file=sys.stderr, flush=True)
        forms["normalize"] = run_normalize_form(dev, 5, not args.no_cpu_baseline)
        print("[bench] normalize form done", file=sys.stderr, flush=True)
        forms["lebesgue"] = run_lebesgue_form(dev, 3, not args.no_cpu_baseline)
        print("[bench] lebesgue form done", file=sys.stderr, flush=True)
        forms["multi"] = run_multi_form(dev, 5, not args.no_cpu_baseline)
        print("[bench] multi form done", file=sys.stderr, flush=True)
        line["forms"] = forms
    print(json.dumps(line))


if __name__ == "__main__":
    main()
