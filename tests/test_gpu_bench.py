"""The bench line end to end on the GPU, at a reduced particle count: one
JSON line with the contract's keys, the roofline and ceiling objects of the
dominant kernel, per-kernel rates, and a repeatable, finite run."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_keeps_the_contract():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
           "--particles-per-species", "20000", "--no-batch", "--no-scan", "--surrogate", "off",
           "--no-cpu-baseline", "--no-fp32-event"]
    print("running:", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and d["unit"] == "site-updates/s" and "workload" in d["config"]
    # value is the whole job's site updates over the timed wall time
    want = 512 * 512 * d["config"]["coupled_steps"] * d["steps"] / (d["ms_per_step"] * 1e-3 * d["steps"])
    assert abs(d["value"] - want) < 1e-6 * want
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] == "hbm" and rf["peak"] == 8000.0 and rf["unit"] == "GB/s"
    assert 0.0 < rf["frac"] < 1.0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    # the live copy ceiling of the library's own kernel, and the kernel against it
    assert 1000.0 < d["stream_ceiling"]["copy_GBps"] < 8000.0
    assert abs(rf["ceiling_frac"] - rf["achieved"] / rf["ceiling"]) < 1e-12
    fs = d["kernels"]["field_step"]
    assert fs["site_updates_per_s"] > d["value"]     # the kernel alone outruns the whole event
    assert d["kernels"]["push"]["particle_steps_per_s"] > d["particle_steps_per_s"]
    assert d["finite"] is True and d["bitwise_repeatable"] is True
    print("bench line: value %.3e, frac %.3f, ceiling frac %.3f" % (d["value"], rf["frac"], rf["ceiling_frac"]))
