"""The autotuner: it times every launch variant, installs the fastest per
(precision, n bucket, m bucket), and a saved table reloads on the same
architecture; results with the tuned variant still meet the parity bars."""
import numpy as np
import pytest
import torch

from oracle import metrics, oracle
from paper_1606_06508_amd import autotune, fh, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_tune_install_save_load(tmp_path):
    n, m = 129, 20000
    try:
        table = autotune.tune([(n, m)], ("fp64", "split"), reps=2, device=DEV)
        for e in table["entries"]:
            assert set(e["all_ms"]) == {str(v[0]) for v in fh.variants(e["precision"])}
            assert e["variant"] == min(e["all_ms"], key=lambda k: e["all_ms"][k]) or \
                e["ms"] == min(e["all_ms"].values())
            assert fh.tune_get(e["precision"], n, m) == e["variant"]
        path = tmp_path / "tune.json"
        autotune.save(table, path)
        for e in table["entries"]:
            assert e["lambda"] == 1
            fh.tune_set(e["precision"], n, m, -1)
        assert autotune.load(path, device=DEV) == len(table["entries"])
        for e in table["entries"]:
            assert fh.tune_get(e["precision"], n, m) == e["variant"]
        g = np.random.default_rng(3)
        nodes = inputs.jittered_nodes(n, g)
        vals = g.standard_normal(n)
        pts = g.uniform(-1, 1, m)
        r_o, lam_o, s_o = oracle.evaluate(nodes, vals, 4, pts)
        t = lambda a: torch.from_numpy(a).to(DEV)  # noqa: E731
        for prec in ("fp64", "split"):
            r, lam = fh.evaluate(t(nodes), t(vals), 4, t(pts), lebesgue=True, precision=prec)
            torch.cuda.synchronize()
            st = metrics.parity(r.cpu().numpy(), lam.cpu().numpy(), r_o, lam_o, s_o,
                                metrics.FP64_LAMBDA_MAX if prec == "fp64" else
                                metrics.SPLIT_LAMBDA_MAX)
            (metrics.check_fp64 if prec == "fp64" else metrics.check_split)(st)
    finally:
        for prec in ("fp64", "split"):
            fh.tune_set(prec, n, m, -1)


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_tune_batch_installs_the_variant_a_new_batch_runs(precision):
    """tune_batch times every batched variant on a batch (one graph launch
    each) and installs the fastest for that batch's shape: a batch created
    afterwards on the same shape runs it, within the oracle's bar."""
    family = "batched_" + precision
    c = inputs.batched_workload(count=64, n_range=(16, 400), m_range=(500, 6000), salt=11)
    n_key, m_key = autotune.batch_key(c["n"]), int(c["m"].sum())
    try:
        table = autotune.tune_batch(c, (precision,), reps=1, device=DEV)
        (e,) = table["entries"]
        assert e["precision"] == family and e["n"] == n_key and e["m"] == m_key
        assert set(e["all_ms"]) == {str(v[0]) for v in fh.variants(family)}
        assert e["ms"] == min(e["all_ms"].values())
        assert fh.tune_get(family, n_key, m_key) == e["variant"]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
        b = fh.Batch(c["n"], c["d"], c["m"], t(c["nodes"]), t(c["values"]), t(c["points"]),
                     precision=precision)
        assert b.variant == e["variant"]
        assert b.strip_points == fh.variant_strip_points(family, e["variant"])
        r = b().cpu().numpy()
        for i in range(0, c["n"].size, 8):
            ns = slice(int(c["node_off"][i]), int(c["node_off"][i + 1]))
            ps = slice(int(c["pt_off"][i]), int(c["pt_off"][i + 1]))
            r_o, lam_o, s_o = oracle.evaluate(c["nodes"][ns], c["values"][ns], int(c["d"][i]),
                                              c["points"][ps])
            st = metrics.parity(r[ps], None, r_o, None, s_o)
            tol = metrics.FP64_TOL if precision == "fp64" else metrics.SPLIT_TOL
            keep = lam_o <= (metrics.FP64_LAMBDA_MAX if precision == "fp64" else
                             metrics.SPLIT_LAMBDA_MAX)
            err = np.abs(r[ps] - r_o)[keep] / s_o[keep]
            assert st["nan_mismatch_r"] == 0 and np.all(err <= tol), (i, st)
        b.close()
    finally:
        fh.tune_set(family, n_key, m_key, -1)


def test_library_loads_a_saved_table(tmp_path):
    """FH_AUTOTUNE_CACHE: the library itself installs a table saved by the
    autotuner on first use (same architecture), with no Python in between;
    its calls then run the saved variants."""
    import json
    import os
    import subprocess
    import sys
    arch = torch.cuda.get_device_properties(DEV).gcnArchName.split(":")[0]
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"arch": arch, "entries": [
        {"precision": "fp64", "n": 1001, "m": 1000000, "lambda": 1, "variant": 3, "ms": 1.0},
        {"precision": "batched_fp64", "n": 300, "m": 50000, "lambda": 0, "variant": 13,
         "ms": 1.0}]}))
    code = ("from paper_1606_06508_amd import fh\n"
            "print(fh.tune_get('fp64', 1001, 10**6), fh.tune_get('batched_fp64', 300, 50000),"
            " fh.tune_get('fp64', 4097, 10**7))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=root, env=dict(os.environ, FH_AUTOTUNE_CACHE=str(path), FH_LOG="1"))
    assert p.returncode == 0, p.stderr
    assert p.stdout.split() == ["3", "13", "25"], (p.stdout, p.stderr)
    assert "2 entries installed" in p.stderr
