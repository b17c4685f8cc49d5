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
