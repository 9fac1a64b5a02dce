"""Host-side checks of bench.py's contract (no GPU): a request for more than one
GPU ends with a message, and the roofline constants are the ones stated."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_constants():
    b = _bench()
    assert b.HBM_PEAK_GBS == 8000.0
    # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz, without packed fp32
    assert abs(b.VALU_F32_PEAK_TFLOPS - 78.6432) < 1e-9
    # populations 2 x 9 x 4 B read and written, phi/Qxx/Qxy read and written
    assert b.ALG_BYTES["step"] == 2 * 9 * 4 * 2 + 3 * 4 * 2
    # the collision's share: populations read and written, phi/Q read; the frozen
    # velocities it writes for the sub-step kernel are overhead of the two-kernel split
    assert b.ALG_BYTES["collide"] == 2 * 9 * 4 * 2 + 3 * 4
    assert b.OVERHEAD_BYTES["collide"] == 4 * 4
    assert b.ALG_BYTES["substeps"] == 3 * 4 * 2
    # observables snapshot: packing 7 x 4 read + 3 x 8 written, five 2D FFTs of two
    # read+write passes over complex64, powers 3 x 8 read + 2 x 4 + 2 x 8 written,
    # shell sums 2 x 4 + 2 x 8 read, defects 2 x 4 read
    assert b.ANALYSIS_BYTES_PER_SITE == (7 * 4 + 3 * 8) + 5 * 2 * 2 * 8 + (3 * 8 + 2 * 4 + 2 * 8) + (2 * 4 + 2 * 8) + 2 * 4


def test_traffic_record_matches_sources_or_is_ignored():
    b = _bench()
    t = b.measured_traffic("collide")
    assert t is None or t > 0
