"""The benchmark's JSON line on the device: a short in-process run of bench.py on
the 2048 x 2048 workload, checked for the fields of its contract and for the
internal consistency of its figures (throughput from the step time, roofline
fractions from achieved / peak, kernel time inside the timed region)."""
import importlib.util
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def run_bench(monkeypatch, capsys, argv):
    b = _bench()
    monkeypatch.setattr(sys, "argv", ["bench.py"] + argv)
    capsys.readouterr()  # only bench.py's own output below
    b.main()
    out = capsys.readouterr().out.strip().splitlines()
    assert len(out) == 1, out
    return b, json.loads(out[0])


def test_bench_line_contract(gpu, monkeypatch, capsys):
    print("case: bench.py --steps 40 --warmup 10 --settle-s 1 --cpu-budget 2 --single-core-budget 2",
          file=sys.__stderr__, flush=True)
    b, d = run_bench(monkeypatch, capsys, ["--steps", "40", "--warmup", "10", "--settle-s", "1", "--cpu-budget", "2",
                                           "--single-core-budget", "2"])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 40 and d["warmup"] == 10
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["dtype"] == "f32"
    assert d["config"]["workload"].startswith("large_2048") and d["config"]["nx"] == d["config"]["ny"] == 2048
    # throughput is sites per step time
    mlups = 2048 * 2048 / (d["ms_per_step"] * 1e-3) / 1e6
    assert abs(mlups - d["value"]) <= 1e-3 * d["value"] + 0.2
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-4
    assert abs(r["achieved"] - r["alg_bytes_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e9) <= 0.01 * r["achieved"]
    if r["traffic"] is not None:  # counters of the same sources: at least the algorithmic bytes
        assert r["traffic"] >= r["alg_bytes_per_launch"]
    # the collision's algorithmic bytes are the populations and the phi/Q read only
    assert r["alg_bytes_per_launch"] == 156 * 2048 * 2048
    assert d["step_roofline"]["alg_bytes_per_site"] == 168
    # kernel durations come from a second pass of the same length with events around
    # every launch; their per-step sum agrees with the event-free timed region
    ks = d["kernel_sum_ms_per_step"]
    assert abs(ks - sum(v[0] for v in d["kernels_ms"].values()) / d["kernel_timing_pass"]["steps"]) < 1e-4
    assert 0.85 * d["ms_per_step"] <= ks <= 1.05 * d["ms_per_step"], (ks, d["ms_per_step"])
    assert d["clock_settle"]["seconds"] == 1 and d["clock_settle"]["untimed_steps"] > 0
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == "MLUPS" and c["value"] > 0 and c["cores"] >= 1
    assert c["single_core"]["cores"] == 1 and c["single_core"]["value"] > 0
    print(f"bench line: {d['value']} MLUPS, collision {r['avg_launch_us']} us ({r['frac']:.3f} of HBM), "
          f"cpu {c['value']} MLUPS", file=sys.__stderr__, flush=True)
