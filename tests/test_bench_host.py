"""Host side of bench.py (no device call): one GPU only, strict JSON output,
and the warm-start entry's books (steps compared over the drops that
converged from both starts)."""
import json
import math
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1906_09530_amd import lbm, warmstart  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_strict_json_replaces_non_finite_numbers():
    obj = {"a": math.nan, "b": [1.0, math.inf, np.float64(-math.inf), 2], "c": {"d": 0.5},
           "e": None, "f": "x", "g": (np.float64(3.0),)}
    out = json.loads(json.dumps(bench.strict_json(obj), allow_nan=False))
    assert out == {"a": None, "b": [1.0, None, None, 2], "c": {"d": 0.5}, "e": None,
                   "f": "x", "g": [3.0]}


def test_column_shape_reports_the_fastest_column_candidate():
    """The autotuner's table mixes column shapes (width > 0) and collision
    variants (width 0); the reported column shape is the fastest of the
    former, whatever the latter's times."""
    table = {(4, 8): 0.61, (16, lbm.COLUMN_STREAM): 0.55, (8, -8): 0.60, (0, 2): 0.45,
             (0, 0): 0.56}
    assert bench.column_shape(table) == [16, lbm.COLUMN_STREAM]
    table[(4, 16)] = 0.50
    assert bench.column_shape(table) == [4, 16]


def test_warm_start_sets_scale_the_radii_consistently():
    """The 512^2-trained set draws training and unseen drops of the same
    absolute radii (those of the 256^2-trained full set's unseen drops)."""
    full, f512 = bench.WARM["full"], bench.WARM["full512"]
    eval_scale_full = full["train_n"] / full["eval_n"]
    assert f512["eval_n"] == full["eval_n"] and f512["eval_r_scale"] == eval_scale_full
    assert f512["train_n"] * f512["train_r_scale"] == full["train_n"]


def test_warm_start_entry_compares_drops_that_converged_from_both(monkeypatch):
    bad = lbm.LBM_E_NONFINITE

    class Net:
        def close(self):
            pass

    def fake_compare(*args, **kw):
        warm = {"steps_warm": [100, 200, 300, 400], "status_warm": [0, 0, 0, bad],
                "fallbacks": 0, "seconds_warm": 1.5, "max_rel_drho": 1e-12,
                "max_abs_dv": 1e-12}
        res = {"inference": "bf16", "reach": kw["reach"], "steps_tanh": [150, 7, 350, 500],
               "status_tanh": [0, bad, 0, 0], "steps_tanh_at_rest": None, "seconds_tanh": 2.0,
               "by_inference": {"bf16": warm}}
        res.update(warm)
        return res

    monkeypatch.setattr(warmstart, "training_set",
                        lambda *a, **k: (np.zeros((4, 7)), np.zeros((4, 3)), {"converged": 4}))
    monkeypatch.setattr(warmstart, "train_network", lambda x, t: (Net(), np.ones(40), 1.0))
    monkeypatch.setattr(warmstart, "compare", fake_compare)
    for which, reach in (("full", 80.0), ("small", None)):
        out = json.loads(json.dumps(bench.strict_json(bench.warmstart_bench(which)),
                                    allow_nan=False))
        assert out["workload"] == "pr" and out["reach"] == reach
        # drops 0 and 2 converged from both starts
        assert out["compared_drops"] == 2
        assert (out["steps_tanh"], out["steps_warm"]) == (500, 400)
        assert out["steps_ratio"] == 0.8
        assert out["status_tanh"] == {"LBM_E_NONFINITE": 1, "LBM_OK": 3}
        assert out["status_warm"] == {"LBM_E_NONFINITE": 1, "LBM_OK": 3}
        assert out["all_converged"] is False
        assert out["by_inference"]["bf16"]["compared_drops"] == 2


def test_cpu_baseline_times_the_oracle_on_the_bench_workload():
    """The cpu_baseline leg: the oracle on the same 1024^2 PR drop, one
    thread and then all cores (OpenMP build), at least one whole step each
    within the budget."""
    out = bench.cpu_baseline(budget_s=0.5)
    assert out["kind"] == "oracle" and out["cores"] >= 1 and out["unit"] == "MLUPS"
    assert 0.0 < out["value"] < 1e3 and 0.0 < out["single_core_value"] < 1e3
    assert "1024x1024 PR drop" in out["sample"]
    json.dumps(out, allow_nan=False)
    one = bench.cpu_baseline(budget_s=0.5, all_cores=False)
    assert one["cores"] == 1
