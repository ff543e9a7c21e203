"""bench.py end to end on the GPU at a small size (5 levels of 64^3): one JSON
line on stdout with every field of its contract, the headline taken as the
fastest variant whose force error matches plain FP64's, the roofline fraction
equal to achieved / peak, per-variant deviations from the FP64 solve of the
same run, and the oracle's CPU timing beside it."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    variants = ["fp64", "fp64_v112", "fp16s_dc_v112", "fp16s_dc+learned"]
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--N", "64", "--steps", "2", "--warmup", "1",
           "--variants", ",".join(variants), "--cpu-sample-cycles", "1"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [x for x in r.stdout.splitlines() if x.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "variants"):
        assert k in d, k
    assert (d["n_gpus"], d["steps"], d["warmup"]) == (1, 2, 1)
    assert d["higher_is_better"] is False and d["unit"] == "ms/solve" and d["data"] == "synthetic"
    assert d["value"] == d["ms_per_step"] > 0
    assert d["config"]["workload"] == "two_plummer_5lev_64"
    assert set(d["variants"]) == set(variants)
    # the headline: the fastest variant at plain FP64's force error
    ok = [v for v, x in d["variants"].items()
          if abs(x["linf_force_error"] - d["variants"]["fp64"]["linf_force_error"])
          <= 5e-3 * d["variants"]["fp64"]["linf_force_error"]]
    assert d["config"]["variant"] in ok
    assert d["value"] == min(d["variants"][v]["ms_per_solve"] for v in ok)
    for v, x in d["variants"].items():
        if v != "fp64":
            assert x["deviation_from_fp64"]["force_rel"] <= 1e-8, v
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-3
    assert rl["traffic"] is None  # the committed counters are for 514^3 only
    assert d["speedup_vs_plain_fp64_same_schedule"] is not None
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
